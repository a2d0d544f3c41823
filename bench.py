#!/usr/bin/env python3
"""Throughput of the concurrent multi-implicit SDC step on one MI355X.

Workload (the 2-D flame of 256 x 256 cells): seeded 9-species / 21-reaction
Arrhenius mechanism, periodic tanh flame 300 -> 2000 K, uniform velocity
1 m/s, dx = 0.01 cm, dt = 5e-5 s, CISDCQ with nu = 1, 5 Gauss-Lobatto nodes,
6 sweeps per step.  A bench step is one full time step (every sweep, every
node: implicit diffusion on one stream, per-cell Newton reaction solves on the
other).  Inputs are resident in device memory before timing starts.

metric: cell-node updates per second per concurrent sweep
        = cells * M * nu * sweeps * steps / timed seconds.
Also reported: Newton iterations per cell-node solve, the roofline of the
dominant kernel (live HIP-event timing inside the library, on the stream the
kernel runs on), the FP64 oracle timed on the host for a sample of the same
workload, and an accuracy gate: one GPU step of the timed workload at its
full size and launch configuration against the oracle's step (<= 1e-8), with
the sweep increments compared in the same norm.  A run with unconverged
solves or a failed gate prints its line with "valid": false and exits 3.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-node updates/s per concurrent-MISDC sweep at 1e-8 rel err; Newton iters/cell"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# algorithmic traffic of one preconditioned CG iteration per unknown, fused:
# read p, q(=Ap), x, r, z/diag and write x, r, z -> 7 doubles
CG_BYTES_PER_UNKNOWN_ITER = 56.0
# algorithmic FP64 work of one Newton iteration for 9 species / 21 reactions
NEWTON_FLOP_PER_ITER_9 = 3.4e3
NEWTON_BYTES_PER_SOLVE_9 = 316.0
# 53 species / 325 reactions: rates ~24k, Jacobian ~13k, LU ~105k, solves ~6k
NEWTON_FLOP_PER_ITER_53 = 1.49e5


def newton_sweep_stats(integ, sweeps):
    """Per-sweep Newton iterations per cell-node solve of the last step:
    mean, p50, p99 and max, from the library's outcome histograms."""
    out = []
    for k in range(sweeps):
        h = integ.newton_histogram(k)
        tot = sum(h[1:])
        if tot == 0:
            out.append({"sweep": k, "solves": 0})
            continue
        cum, pct = 0, {}
        for v in range(1, len(h)):
            cum += h[v]
            for q in (0.5, 0.99):
                if q not in pct and cum >= q * tot:
                    pct[q] = v
        out.append({"sweep": k, "solves": sum(h), "failed": h[0],
                    "mean": sum(v * h[v] for v in range(1, len(h))) / tot,
                    "p50": pct[0.5], "p99": pct[0.99],
                    "max": max(v for v in range(1, len(h)) if h[v])})
    return out


def measured_traffic(profile_name, source_rel):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", profile_name)
    try:
        text = open(path).read()
        sha = re.search(r"source_sha1: ([0-9a-f]+)", text).group(1)
        val = float(re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text).group(1))
        cur = hashlib.sha1(open(os.path.join(ROOT, source_rel), "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    return val if cur == sha else None


def measured_fp64_ops(kernel, source_rel):
    """FP64 lane operations per launch of a kernel from the committed
    rocprofv3 FLOP-counter summary, or None when the kernel source has
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "pmc_fp64_ops_flame2d_256.md")
    try:
        text = open(path).read()
        m = re.search(r"fp64_ops_per_launch: " + re.escape(kernel) +
                      r": ([0-9.eE+]+) source_sha1: ([0-9a-f]+)", text)
        val, sha = float(m.group(1)), m.group(2)
        cur = hashlib.sha1(open(os.path.join(ROOT, source_rel), "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    return val if cur == sha else None


def fp64_counter_rates(d_ms, d_n, r_ms, r_n, spec):
    """Counted FP64 lane operations of the two leaves against the FP64 vector
    peak, with this run's average launch durations (``spec``: the reaction
    solve is the kernel generated for the mechanism)."""
    out = {}
    reaction = (("newton_spec", "paper_1801_01201_amd/csrc/chem_spec.cpp") if spec else
                ("newton_kernel<9, true>", "paper_1801_01201_amd/csrc/chem.hip"))
    for kernel, src, ms, cnt in (("cg_tile_kernel<9, 1>", "paper_1801_01201_amd/csrc/cg.hip", d_ms, d_n),
                                 reaction + (r_ms, r_n)):
        ops = measured_fp64_ops(kernel, src)
        if ops is None or cnt == 0:
            out[kernel] = None
            continue
        tf = ops / (ms / cnt * 1e-3) / 1e12
        out[kernel] = {"ops_per_launch": ops, "tflops": tf,
                       "frac_of_fp64_peak": tf / FP64_VECTOR_PEAK_TFLOPS}
    return out


def overlap_probe():
    """Eager steps, a pause, then graph-replayed steps of the 256x256 workload."""
    import time
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import Mechanism, Grid, Integrator, initial_state
    native.lib()
    cfg = workload()
    mech = synth.make_mechanism(**cfg["mech"])
    nx, ny = cfg["n"]
    mh = Mechanism(mech)
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    state, _ = initial_state(mh, torch.tensor(Y.reshape(9, -1), device="cuda"),
                             torch.tensor(T.ravel(), device="cuda"))
    for graph in (False, True):
        integ = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"],
                           scheme=cfg["scheme"], use_graph=graph)
        s = state.clone()
        for _ in range(2):
            integ.step(s, cfg["dt"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            integ.step(s, cfg["dt"])
        torch.cuda.synchronize()
        print(json.dumps({"execution": "graph" if graph else "eager",
                          "ms_per_step": (time.perf_counter() - t0) / 3 * 1e3}), flush=True)
        integ.close()
        time.sleep(0.3)
    g.close()


def analyse_trace(directory):
    """Per phase of a kernel trace (phases split at gaps of more than 100 ms):
    busy time of the diffusion kernels (cg_*, cyclic_*, tridiagonal and
    diffusion solves) and of the reaction kernels (newton*), and the time both
    run at once."""
    import csv
    import glob
    paths = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if not paths:
        print(f"no kernel trace under {directory}", file=sys.stderr)
        sys.exit(1)
    rows = list(csv.DictReader(open(paths[0])))
    ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)

    def merged(iv):
        out = []
        for a, b in sorted(iv):
            if out and a <= out[-1][1]:
                out[-1][1] = max(out[-1][1], b)
            else:
                out.append([a, b])
        return out

    def busy(iv):
        return sum(b - a for a, b in iv)

    def both(x, y):
        tot = i = j = 0
        while i < len(x) and j < len(y):
            lo, hi = max(x[i][0], y[j][0]), min(x[i][1], y[j][1])
            tot += max(0, hi - lo)
            if x[i][1] < y[j][1]:
                i += 1
            else:
                j += 1
        return tot

    phases, cur = [], [ks[0]]
    for k in ks[1:]:
        if k[0] - cur[-1][1] > 100_000_000:
            phases.append(cur)
            cur = []
        cur.append(k)
    phases.append(cur)
    diff_keys = ("cg_", "cyclic", "tridiag", "diffusion")
    for n, ph in enumerate(phases):
        d = merged([(a, b) for a, b, k in ph if any(t in k for t in diff_keys)])
        r = merged([(a, b) for a, b, k in ph if "newton" in k])
        print(json.dumps({"phase": n, "kernels": len(ph), "span_ms": (ph[-1][1] - ph[0][0]) / 1e6,
                          "diffusion_busy_ms": busy(d) / 1e6, "reaction_busy_ms": busy(r) / 1e6,
                          "overlap_ms": both(d, r) / 1e6}))


def workload():
    import synth
    c = synth.config("flame2d_256")
    return c


def host_description():
    """CPU model and the cores this process may use (for the CPU baseline)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _oracle_sample(cfg, nx, ny, sweeps):
    """Wall and CPU seconds of the oracle's step (``sweeps`` sweeps) on an
    nx x ny version of the workload, and the cell-node updates it made."""
    import synth
    from oracle.adr import FlameProblem, relaxed_initial_state
    from oracle.sdc import sdc_step
    mech = synth.make_mechanism(**cfg["mech"])
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    prob = FlameProblem(mech, cfg["dx"], cfg["u"])
    phi = relaxed_initial_state(prob, Y, T)
    nu_tol = cfg.get("nu_tol", 0.0)
    ps = []
    w0, c0 = time.perf_counter(), time.process_time()
    sdc_step(prob, phi, cfg["dt"], cfg["n_nodes"], sweeps, cfg["scheme"], nu=cfg["nu"],
             nu_tol=nu_tol if nu_tol > 0 else None, passes=ps)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    M = cfg["n_nodes"] - 1
    return wall, cpu, nx * ny * M * (sum(ps) if ps else cfg["nu"] * sweeps)


def cpu_baseline_leg(cfg):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    the same flame, mechanism, step and scheme on 128 x 128 cells (a quarter
    of the cells) for three sweeps, with the threads it takes by itself (its
    per-field diffusion systems in parallel, NumPy's own threading), and
    once more on 64 x 64 cells with every thread pool limited to one."""
    from threadpoolctl import threadpool_limits
    import oracle.transport as otr
    wall, cpu, updates = _oracle_sample(cfg, 128, 128, 3)
    saved = otr.SOLVE_THREADS
    try:
        otr.SOLVE_THREADS = 1
        with threadpool_limits(limits=1):
            w1, _, u1 = _oracle_sample(cfg, 64, 64, 3)
    finally:
        otr.SOLVE_THREADS = saved
    M = cfg["n_nodes"] - 1
    out = {"value": updates / wall, "unit": "cell-node updates/s",
           "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
           "sample": f"3 CISDCQ-{cfg['nu']} sweeps ({M} nodes) of the same flame workload on "
                     f"128x128 cells (one quarter of the cells), wall {wall:.1f} s, CPU "
                     f"{cpu:.1f} s; the metric is per cell-node update",
           "seconds": wall,
           "one_thread": {"value": u1 / w1, "sample": "3 sweeps on 64x64 cells, every thread "
                                                       f"pool limited to one, wall {w1:.1f} s"}}
    out.update(host_description())
    return out


def accuracy_gate(cfg, mech, mh, state0, tune):
    """The timed workload at its full size and launch configuration: one GPU
    step from the benchmark's initial state against the oracle's step from
    the same synthetic input (field-normalised max error <= 1e-8), and the
    GPU's sweep increments against the oracle's in the same norm."""
    import numpy as np
    import synth
    from oracle.adr import FlameProblem, relaxed_initial_state
    from oracle.sdc import sdc_step
    from paper_1801_01201_amd.flame import Grid, Integrator
    nx, ny = cfg["n"]
    nu_tol = cfg.get("nu_tol", 0.0)
    st = state0.clone()
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    integ = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"],
                       scheme=cfg["scheme"], nu_tol=nu_tol, cg_rtol=cfg.get("cg_rtol", 1e-13),
                       pipeline=cfg.get("pipeline", False))
    if tune:
        integ.set_tune(tune["cg_variant"], tune["cg_blocks"], tune["cyclic"], tune["serialize"],
                       tune["cu_split"], tune["stagger"], tune.get("fused", 0))
    integ.step(st, cfg["dt"])
    out = st.cpu().numpy()
    s = integ.stats()
    integ.close()
    g.close()
    print(f"[bench] gate: GPU step done, oracle step on {nx}x{ny} follows", file=sys.stderr,
          flush=True)
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    prob = FlameProblem(mech, cfg["dx"], cfg["u"])
    ps, fi = [], []

    def progress(k, inc):
        print(f"[bench] gate: oracle sweep {k} done", file=sys.stderr, flush=True)

    w0 = time.perf_counter()
    ref, _ = sdc_step(prob, relaxed_initial_state(prob, Y, T), cfg["dt"], cfg["n_nodes"],
                      cfg["sweeps"], cfg["scheme"], nu=cfg["nu"],
                      nu_tol=nu_tol if nu_tol > 0 else None, passes=ps, field_increments=fi,
                      progress=progress)
    wall = time.perf_counter() - w0
    ref = ref.reshape(10, -1)
    err = float((np.abs(out - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())
    inc_ref = [float((f[:, 0] / f[:, 1]).max()) for f in fi]
    inc_err = max(abs(a - b) for a, b in zip(s["sweep_increment"], inc_ref))
    ok = (err <= 1e-8 and s["converged"] and len(inc_ref) == len(s["sweep_increment"])
          and (nu_tol <= 0 or s["nested_passes"] == ps))
    return {"err": err, "tol": 1e-8, "passed": bool(ok), "grid": f"{nx}x{ny}",
            "launch_config": tune, "sweep_increment_gpu": s["sweep_increment"],
            "sweep_increment_oracle": inc_ref, "sweep_increment_max_abs_diff": inc_err,
            "nested_passes": s["nested_passes"], "oracle_seconds": wall}


def timed_leg(mh, g, cfg, state, args, tune, use_graph):
    """The timed steps from ``state`` (not modified) with a fresh integrator in
    the tuned launch configuration, issued eagerly or replayed as one captured
    HIP graph per step, without kernel timing events (those are not recorded
    in graphs; the roofline comes from the profiled steps)."""
    import torch
    from paper_1801_01201_amd.flame import Integrator
    gi = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"],
                    scheme=cfg["scheme"], use_graph=use_graph, cg_rtol=cfg.get("cg_rtol", 1e-13),
                    serialize=args.serialize, pipeline=cfg.get("pipeline", False))
    if tune:
        gi.set_tune(tune["cg_variant"], tune["cg_blocks"], tune["cyclic"], tune["serialize"],
                    tune["cu_split"], tune["stagger"], tune.get("fused", 0))
    st = state.clone()
    for _ in range(max(1, args.warmup)):
        gi.step(st, cfg["dt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gi.step(st, cfg["dt"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s = gi.stats()
    gi.close()
    nx, ny = cfg["n"]
    upd = nx * ny * (cfg["n_nodes"] - 1) * cfg["nu"] * cfg["sweeps"] * args.steps
    return {"value": upd / el, "ms_per_step": el / args.steps * 1e3,
            "newton_failed": s["newton_failed"], "cg_failed": s["cg_failed"],
            "converged": s["converged"]}


def ensemble_main(args):
    """64 independent periodic 1-D flames of 128..4096 cells with a 10x
    spread of step sizes (3 Gauss-Lobatto nodes, 4 sweeps, CISDCQ-1); every
    step of every flame in one call, per-flame dt, autotuned.  The same steps
    are timed replayed as one HIP graph per step and issued eagerly; the
    faster of the two is the throughput (``execution`` names it), and a third,
    eager leg with kernel timing gives the roofline of the dominant kernel."""
    import numpy as np
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import Mechanism, Grid, Integrator, initial_state
    native.lib()
    cfg = synth.config("ensemble64")
    mech = synth.make_mechanism(**cfg["mech"])
    lengths, dts, flames = synth.ensemble_flames(mech, cfg["n_flames"], cfg["len_range"], cfg["dt"],
                                                 cfg["dt_spread"], cfg["dx"][0], cfg["ens_seed"])
    nf = len(lengths)
    n = int(np.sum(lengths))
    M = cfg["n_nodes"] - 1
    mh = Mechanism(mech)
    g = Grid(ensemble=(lengths, [cfg["dx"][0]] * nf, [cfg["u"][0]] * nf))
    Y = np.concatenate([f[0] for f in flames], axis=1)
    T = np.concatenate([f[1] for f in flames])
    state, _ = initial_state(mh, torch.tensor(Y, device="cuda"), torch.tensor(T, device="cuda"))
    d_dt = torch.tensor(dts, dtype=torch.float64, device="cuda")
    kw = dict(n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"], scheme=cfg["scheme"])
    res = {}
    tune = None
    for mode in ("graph", "eager", "profile"):
        integ = Integrator(mh, g, use_graph=(mode == "graph"), profile=(mode == "profile"), **kw)
        if tune is None and args.tune:
            integ.set_tune(*[int(v) for v in args.tune.split(",")])
            tune = integ.tune()
        elif tune is None and not args.no_autotune:
            tune = integ.autotune(state, 0.0, dt_per_flame=d_dt, reps=3)
        elif tune is not None:
            integ.set_tune(tune["cg_variant"], tune["cg_blocks"], tune["cyclic"], tune["serialize"],
                           tune["cu_split"], tune["stagger"], tune.get("fused", 0))
        st = state.clone()
        for _ in range(max(1, args.warmup)):
            integ.step(st, 0.0, dt_per_flame=d_dt)
        torch.cuda.synchronize()
        native.misdc_reset_profile(integ.handle)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            integ.step(st, 0.0, dt_per_flame=d_dt)
        torch.cuda.synchronize()
        res[mode] = (time.perf_counter() - t0, integ.stats(),
                     newton_sweep_stats(integ, cfg["sweeps"]))
        integ.close()
    execution = "graph" if res["graph"][0] <= res["eager"][0] else "eager"
    el, stats, newton_sweeps = res[execution]
    elp, sp, _ = res["profile"]
    updates = n * M * cfg["nu"] * cfg["sweeps"] * args.steps
    d_ms, d_n = sp["diffusion_kernel_ms"], sp["diffusion_kernel_launches"]
    r_ms, r_n = sp["newton_kernel_ms"], sp["newton_kernel_launches"]
    newton_per_cell = sp["newton_iters"] / max(1, sp["newton_solves"])
    if d_ms >= r_ms:
        avg_s = d_ms / max(1, d_n) * 1e-3
        # one solve reads rhs and writes y for 9 fields, reads the face
        # coefficients once: 2 * 9 * 8 + 8 bytes per cell
        byts = (2 * 9 * 8 + 8) * n
        roof = {"kernel": "cyclic_wave_kernel (one wavefront per periodic tridiagonal system)",
                "bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": byts / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": avg_s * 1e3, "launches": d_n,
                "algorithmic_bytes_per_launch": byts}
    elif tune and tune.get("fused"):
        # one persistent launch per stage: the flames' tridiagonal systems and
        # the cells' Newton solves from one work queue; achieved counts the
        # reaction solve's FP64 work only (the diffusion systems add little)
        avg_s = r_ms / max(1, r_n) * 1e-3
        flops = NEWTON_FLOP_PER_ITER_9 * n * newton_per_cell
        roof = {"kernel": "stage_kernel (fused stage: tridiagonal systems and per-cell Newton "
                          "solves from one atomic work queue)", "bound": "alu",
                "achieved": flops / avg_s / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / avg_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": None, "avg_launch_ms": avg_s * 1e3, "launches": r_n}
    else:
        avg_s = r_ms / max(1, r_n) * 1e-3
        flops = NEWTON_FLOP_PER_ITER_9 * n * newton_per_cell
        roof = {"kernel": "newton_kernel<9> (per-cell reaction solve)", "bound": "alu",
                "achieved": flops / avg_s / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / avg_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": None, "avg_launch_ms": avg_s * 1e3, "launches": r_n}
    line = {
        "metric": METRIC, "value": updates / el, "unit": "cell-node updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble64: {nf} periodic 1-D flames of "
                               f"{int(lengths.min())}..{int(lengths.max())} cells ({n} cells), "
                               f"per-flame dt {dts.min():.3g}..{dts.max():.3g} s, "
                               f"CISDCQ-{cfg['nu']}, {cfg['n_nodes']} nodes, {cfg['sweeps']} sweeps",
                   "cells": n, "flames": nf},
        "newton_iters_per_cell": newton_per_cell,
        "newton_iters_per_sweep": newton_sweeps,
        "execution": execution,
        "graph_ms_per_step": res["graph"][0] / args.steps * 1e3,
        "eager_ms_per_step": res["eager"][0] / args.steps * 1e3,
        "eager_profiled_ms_per_step": elp / args.steps * 1e3,
        "roofline": roof,
        "kernel_split": {"diffusion_solve_ms_per_launch": d_ms / max(1, d_n),
                         "newton_ms_per_launch": r_ms / max(1, r_n),
                         "diffusion_solve_share_of_step": d_ms / (elp * 1e3),
                         "newton_share_of_step": r_ms / (elp * 1e3)},
        "autotune": tune,
        "newton_failed": stats["newton_failed"],
    }
    mh.close()
    print(json.dumps(line), flush=True)


def n53_main(args):
    """The 53-species / 325-reaction flame on 512 x 512 cells (CISDCQ-1,
    5 nodes, 6 sweeps, dt 2.5e-5 s): the reaction solve runs one wavefront
    per cell, the implicit diffusion of 53 fields runs the CG kernel with
    vectors in global memory.  Both Newton LU variants are timed (FP64 LU;
    FP32 LU on the matrix cores refined in FP64); ``value`` is the one named
    by --lu.  Eager steps with kernel timing (roofline of the dominant
    kernel)."""
    import numpy as np
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import Mechanism, Grid, Integrator, initial_state
    native.lib()
    cfg = synth.config("flame2d_512_n53")
    mech = synth.make_mechanism(**cfg["mech"])
    N = mech["N"]
    nx, ny = cfg["n"]
    n = nx * ny
    M = cfg["n_nodes"] - 1
    mh = Mechanism(mech)
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    state, _ = initial_state(mh, torch.tensor(Y.reshape(N, -1), device="cuda"),
                             torch.tensor(T.ravel(), device="cuda"))
    torch.cuda.synchronize()
    print("[bench] n53: initial state ready", file=sys.stderr, flush=True)
    runs = {}
    for lu in ("fp64", "fp32_mfma"):
        integ = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"],
                           scheme=cfg["scheme"], profile=True,
                           newton=native.newton_opts(lu=lu))
        st = state.clone()
        for _ in range(args.warmup):
            integ.step(st, cfg["dt"])
        torch.cuda.synchronize()
        native.misdc_reset_profile(integ.handle)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            integ.step(st, cfg["dt"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stats = integ.stats()
        stats["per_sweep"] = newton_sweep_stats(integ, cfg["sweeps"])
        integ.close()
        runs[lu] = (el, stats, st)
        print(f"[bench] n53 {lu}: {el / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    el, stats, st = runs[args.lu]
    a64, a32 = runs["fp64"][2], runs["fp32_mfma"][2]
    agree = float(((a64 - a32).abs().amax(dim=1) / a64.abs().amax(dim=1).clamp_min(1e-300)).max())
    updates = n * M * cfg["nu"] * cfg["sweeps"] * args.steps
    d_ms, d_n = stats["diffusion_kernel_ms"], stats["diffusion_kernel_launches"]
    r_ms, r_n = stats["newton_kernel_ms"], stats["newton_kernel_launches"]
    newton_per_cell = stats["newton_iters"] / max(1, stats["newton_solves"])
    cg_per_solve = stats["cg_iters"] / max(1, stats["cg_solves"])
    if d_ms >= r_ms:
        avg_s = d_ms / max(1, d_n) * 1e-3
        byts = CG_BYTES_PER_UNKNOWN_ITER * N * n * cg_per_solve
        roof = {"kernel": "cg_kernel (Jacobi-PCG, vectors in global memory, 53 fields)",
                "bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": byts / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": avg_s * 1e3, "launches": d_n,
                "algorithmic_bytes_per_launch": byts, "cg_iterations_per_launch": cg_per_solve}
    else:
        avg_s = r_ms / max(1, r_n) * 1e-3
        flops = NEWTON_FLOP_PER_ITER_53 * n * newton_per_cell
        roof = {"kernel": f"newton_wave_kernel (one wavefront per cell, LU {args.lu})",
                "bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / avg_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": None, "avg_launch_ms": avg_s * 1e3, "launches": r_n}
    variants = {}
    for lu, (e, s2, _) in runs.items():
        variants[lu] = {"ms_per_step": e / args.steps * 1e3,
                        "newton_ms_per_launch": s2["newton_kernel_ms"] / max(1, s2["newton_kernel_launches"]),
                        "newton_iters_per_cell": s2["newton_iters"] / max(1, s2["newton_solves"]),
                        "fp32_solves": s2["newton_lu_solves"],
                        "fp64_fallbacks": s2["newton_lu_fallbacks"],
                        "newton_failed": s2["newton_failed"]}
    line = {
        "metric": METRIC, "value": updates / el, "unit": "cell-node updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"flame2d_512_n53: 2-D periodic {nx}x{ny} flame, {N} species / "
                               f"{mech['R']} reactions, CISDCQ-{cfg['nu']}, {cfg['n_nodes']} nodes, "
                               f"{cfg['sweeps']} sweeps, dt {cfg['dt']} s, Newton LU {args.lu}",
                   "cells": n},
        "newton_iters_per_cell": newton_per_cell,
        "newton_iters_per_sweep": stats["per_sweep"],
        "cg_iters_per_solve": cg_per_solve,
        "roofline": roof,
        "kernel_split": {"diffusion_solve_ms_per_launch": d_ms / max(1, d_n),
                         "newton_ms_per_launch": r_ms / max(1, r_n),
                         "diffusion_solve_share_of_step": d_ms / (el * 1e3),
                         "newton_share_of_step": r_ms / (el * 1e3)},
        "lu_variants": variants,
        "fp32_vs_fp64_state_difference": agree,
        "newton_failed": stats["newton_failed"], "cg_failed": stats["cg_failed"],
    }
    mh.close()
    print(json.dumps(line), flush=True)


def mlp_main(args):
    """The 256 x 256 flame with the learned Newton guess: the network
    (11 -> 256 -> 256 -> 10, BF16 operands, FP32 accumulation) is trained on
    the GPU on the reaction problems recorded from one step of each of four
    independent flames (initial-condition seeds 200..203) plus their
    cold-start relaxation problems, then the benchmark's flame (held out) is
    stepped with and without it.  Reported: step throughput with the guess,
    Newton iterations per cell both ways, the cold-start relaxation with
    and without the guess, and the training throughput."""
    import numpy as np
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import (Mechanism, Grid, Integrator, initial_state, GuessNet,
                                            RELAX_TIME)
    from paper_1801_01201_amd.guess import pack_params, record_problems, train
    native.lib()
    cfg = synth.config("flame2d_256")
    mech = synth.make_mechanism(**cfg["mech"])
    nx, ny = cfg["n"]
    n = nx * ny
    M = cfg["n_nodes"] - 1
    mh = Mechanism(mech)
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    kw = dict(n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"], scheme=cfg["scheme"])

    def relax_problem(Y, T):
        b = torch.tensor(Y.reshape(9, -1), device="cuda")
        h = torch.empty(n, dtype=torch.float64, device="cuda")
        native.misdc_enthalpy(mh.handle, n, b, torch.tensor(T.ravel(), device="cuda"), h)
        return b, h, torch.full((n,), RELAX_TIME, dtype=torch.float64, device="cuda")

    # training data: sweep problems + relaxation problems of four flames
    t0 = time.perf_counter()
    states, rb, rh, rc, rY = [], [], [], [], []
    for seed in (200, 201, 202, 203):
        Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"], seed=seed)
        b, h, c = relax_problem(Y, T)
        Yo = b.clone()
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        native.misdc_reaction_solve_batch(mh.handle, n, b, h, c, Yo, None, None, it)
        rb.append(b), rh.append(h), rc.append(c), rY.append(Yo)
        st, _ = initial_state(mh, b, torch.tensor(T.ravel(), device="cuda"))
        states.append(st)
    bY, hh, cc, Ys = record_problems(mh, g, states, cfg["dt"], **kw)
    bY = torch.cat([bY] + rb, dim=1).contiguous()
    hh = torch.cat([hh] + rh).contiguous()
    cc = torch.cat([cc] + rc).contiguous()
    Ys = torch.cat([Ys] + rY, dim=1).contiguous()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_train = hh.numel()
    print(f"[bench] mlp: {n_train} training problems in {t_data:.1f} s", file=sys.stderr, flush=True)
    net = GuessNet(9, 256, "bf16")
    net.set_params(pack_params(synth.mlp_init(net.sizes, 7)))
    epochs, batch = 4, 65536
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(mh, net, bY, hh, cc, Ys, epochs=epochs, batch=batch, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    samples = (n_train // batch) * batch * epochs
    flop_per_sample = 3 * 2 * sum(a * b for a, b in zip(net.sizes[:-1], net.sizes[1:]))
    print(f"[bench] mlp: trained {epochs} epochs in {t_train:.2f} s, loss {hist}",
          file=sys.stderr, flush=True)
    del bY, hh, cc, Ys, states
    # held-out benchmark flame: cold-start relaxation and steps, both guesses
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    b, h, c = relax_problem(Y, T)
    relax = {}
    for name in ("plain", "learned"):
        Yo = b.clone()
        if name == "learned":
            native.misdc_reaction_guess_mlp(mh.handle, net.handle, n, b, h, c, Yo)
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        native.misdc_reaction_solve_batch(mh.handle, n, b, h, c, Yo, None, None, it)
        relax[name] = float(it.double().mean())
    state, _ = initial_state(mh, b, torch.tensor(T.ravel(), device="cuda"))
    res = {}
    for name in ("plain", "learned"):
        integ = Integrator(mh, g, **kw)
        if name == "learned":
            integ.set_guess(net, sweeps=args.guess_sweeps)
        st = state.clone()
        for _ in range(args.warmup):
            integ.step(st, cfg["dt"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            integ.step(st, cfg["dt"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s = integ.stats()
        integ.close()
        res[name] = (el, s, st)
    el, s, st = res["learned"]
    diff = float(((res["plain"][2] - st).abs().amax(dim=1) /
                  res["plain"][2].abs().amax(dim=1)).max())
    updates = n * M * cfg["nu"] * cfg["sweeps"] * args.steps
    line = {
        "metric": METRIC, "value": updates / el, "unit": "cell-node updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "flame2d_256_mlp: the 256x256 flame (CISDCQ-1, 5 nodes, 6 sweeps) "
                               "with the learned Newton guess (11->256->256->10, bf16 MFMA, "
                               "trained on the GPU on four independent flames)", "cells": n},
        "newton_iters_per_cell": {k: v[1]["newton_iters"] / max(1, v[1]["newton_solves"])
                                  for k, v in res.items()},
        "ms_per_step_plain_guess": res["plain"][0] / args.steps * 1e3,
        "guess_sweeps": args.guess_sweeps,
        "learned_guess_taken": s["newton_guess_learned"],
        "newton_solves": s["newton_solves"],
        "state_difference_vs_plain_guess": diff,
        "cold_start_relaxation_newton_iters_per_cell": relax,
        "training": {"problems": n_train, "epochs": epochs, "batch": batch,
                     "seconds": t_train, "samples_per_s": samples / t_train,
                     "gemm_tflops": samples * flop_per_sample / t_train / 1e12,
                     "bf16_mfma_peak_tflops": 2500.0, "loss_per_epoch": [float(v) for v in hist],
                     "data_seconds": t_data},
        "newton_failed": s["newton_failed"], "cg_failed": s["cg_failed"],
    }
    net.close()
    mh.close()
    print(json.dumps(line), flush=True)


def rnu_main(args):
    """The paper's cost ratio R_nu measured in time on the 256x256 flame: each
    scheme sweeps (misdc_sweep) until its sweep increment is at most
    --rnu-tol, then a step of that many sweeps is timed; R_nu = t(MISDCQ) /
    t(CISDCQ-nu).  MISDCQ runs its D and R tasks in turn (its dependencies
    leave nothing to overlap), CISDCQ-nu on the two streams."""
    import numpy as np
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import Mechanism, Grid, Integrator, initial_state
    native.lib()
    cfg = synth.config(args.rnu_base)
    mech = synth.make_mechanism(**cfg["mech"])
    N = mech["N"]
    nx, ny = cfg["n"]
    n = nx * ny
    mh = Mechanism(mech)
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    state, _ = initial_state(mh, torch.tensor(Y.reshape(N, -1), device="cuda"),
                             torch.tensor(T.ravel(), device="cuda"))
    torch.cuda.synchronize()
    runs = {}
    for name, scheme, nu in (("MISDCQ", "misdcq", 1), ("CISDCQ-1", "cisdcq", 1),
                             ("CISDCQ-2", "cisdcq", 2), ("CISDCQ-3", "cisdcq", 3)):
        probe = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=1, nu=nu, scheme=scheme)
        st = state.clone()
        probe.begin(st, cfg["dt"])
        incs = []
        while len(incs) < 64:
            probe.sweep()
            incs.append(probe.stats()["sweep_increment"][-1])
            if incs[-1] <= args.rnu_tol:
                break
        probe.end()
        probe.close()
        K = len(incs)
        integ = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=K, nu=nu, scheme=scheme)
        st = state.clone()
        for _ in range(max(1, args.warmup)):
            integ.step(st, cfg["dt"])
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            st = state.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            integ.step(st, cfg["dt"])
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        integ.close()
        runs[name] = {"sweeps": K, "ms_per_step": float(np.median(ts)) * 1e3,
                      "final_increment": incs[-1], "converged": incs[-1] <= args.rnu_tol}
        print(f"[bench] rnu {name}: {K} sweeps, {runs[name]['ms_per_step']:.2f} ms",
              file=sys.stderr, flush=True)
    base = runs["MISDCQ"]["ms_per_step"]
    ratios = {k: base / v["ms_per_step"] for k, v in runs.items() if k != "MISDCQ"}
    best = max(ratios, key=ratios.get)
    M = cfg["n_nodes"] - 1
    line = {
        "metric": "R_nu = time of MISDCQ / time of CISDCQ-nu to reach the sweep-increment "
                  "tolerance", "value": ratios[best], "unit": "ratio", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs[best]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"flame2d_256_rnu ({args.rnu_base}): 2-D periodic {nx}x{ny} "
                               f"flame, {N} species / {mech['R']} reactions, "
                               f"{cfg['n_nodes']} Gauss-Lobatto nodes, dt "
                               f"{cfg['dt']} s, sweeps until the increment is <= {args.rnu_tol}",
                   "cells": n, "best": best},
        "R_nu": ratios, "runs": runs,
        "cell_node_updates_per_s": {k: n * M * v["sweeps"] * (int(k[-1]) if k != "MISDCQ" else 1)
                                    / (v["ms_per_step"] * 1e-3) for k, v in runs.items()},
    }
    g.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true")
    ap.add_argument("--nu", type=int, default=None)
    ap.add_argument("--sweeps", type=int, default=None)
    ap.add_argument("--cg-rtol", type=float, default=1e-13,
                    help="relative residual of the implicit diffusion solves (the accuracy gate "
                         "runs with the same value)")
    ap.add_argument("--nu-tol", type=float, default=0.0,
                    help="adaptive nested iterations (CISDCQ, --nu >= 3 passes at most): a "
                         "sweep stops after pass l >= 2 once that pass changed the state by at "
                         "most nu_tol times the first pass's change")
    ap.add_argument("--serialize", action="store_true")
    ap.add_argument("--pipeline", action="store_true",
                    help="pipelined nested iterations (CISDCQ, --nu >= 2): the tasks of each "
                         "pass on streams of their own")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune", default=None,
                    help="launch configuration instead of autotuning: cg_variant,cg_blocks,"
                         "cyclic,serialize,cu_split,stagger")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the extra timing of the same steps replayed as one HIP graph")
    ap.add_argument("--workload", default="flame2d_256",
                    choices=["flame2d_256", "ensemble64", "flame2d_512_n53", "flame2d_256_mlp",
                             "flame2d_256_rnu"])
    ap.add_argument("--rnu-tol", type=float, default=1e-8,
                    help="flame2d_256_rnu: sweeps continue until the sweep increment is below this")
    ap.add_argument("--rnu-base", default="flame2d_256", choices=["flame2d_256", "flame2d_512_n53"],
                    help="flame2d_256_rnu: the workload whose schemes are compared")
    ap.add_argument("--guess-sweeps", type=int, default=1,
                    help="flame2d_256_mlp: leading sweeps that use the learned guess (0: all)")
    ap.add_argument("--lu", default="fp64", choices=["fp64", "fp32_mfma"],
                    help="flame2d_512_n53: precision of the Newton LU of the timed run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device 4 times (calibrates the HBM "
                         "byte counters of rocprofv3 --pmc) and exit")
    ap.add_argument("--overlap-probe", action="store_true",
                    help="only run 2 + 3 eager steps, a pause, then 2 + 3 graph-replayed steps "
                         "of the 256x256 workload (default launch configuration), for a kernel "
                         "trace that shows the overlap of the two solves in each; then exit")
    ap.add_argument("--analyse-trace", default=None, metavar="DIR",
                    help="only read a rocprofv3 kernel trace (CSV) under DIR and print, per "
                         "phase, the busy time of the diffusion and reaction kernels and "
                         "their overlap; then exit")
    args = ap.parse_args()
    if args.analyse_trace:
        return analyse_trace(args.analyse_trace)
    if args.overlap_probe:
        return overlap_probe()
    if args.copy_calibration:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": src.numel() * 8, "copies": 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              f"path (spatial slabs, halo exchange, all-reduces) is not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ensemble64":
        return ensemble_main(args)
    if args.workload == "flame2d_512_n53":
        return n53_main(args)
    if args.workload == "flame2d_256_rnu":
        return rnu_main(args)
    if args.workload == "flame2d_256_mlp":
        return mlp_main(args)
    cfg = workload()
    if args.nu:
        cfg["nu"] = args.nu
    if args.sweeps:
        cfg["sweeps"] = args.sweeps
    cfg["nu_tol"] = args.nu_tol
    cfg["cg_rtol"] = args.cg_rtol
    cfg["pipeline"] = args.pipeline
    # the CPU leg runs first, before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline_leg(cfg)
    if cpu:
        print(f"[bench] cpu baseline: {cpu['value']:.4g} {cpu['unit']} ({cpu['sample']})",
              file=sys.stderr, flush=True)

    import numpy as np
    import torch
    import synth
    from paper_1801_01201_amd import native
    from paper_1801_01201_amd.flame import Mechanism, Grid, Integrator, initial_state
    native.lib()
    mech = synth.make_mechanism(**cfg["mech"])
    nx, ny = cfg["n"]
    n = nx * ny
    M = cfg["n_nodes"] - 1
    mh = Mechanism(mech)
    g = Grid(2, [nx, ny], list(cfg["dx"]), list(cfg["u"]))
    Y, T = synth.flame_2d(mech, nx, ny, *cfg["dx"])
    state, _ = initial_state(mh, torch.tensor(Y.reshape(9, -1), device="cuda"),
                             torch.tensor(T.ravel(), device="cuda"))
    state_init = state.clone()
    integ = Integrator(mh, g, n_nodes=cfg["n_nodes"], sweeps=cfg["sweeps"], nu=cfg["nu"],
                       scheme=cfg["scheme"], serialize=args.serialize, profile=True,
                       nu_tol=args.nu_tol, cg_rtol=args.cg_rtol, pipeline=args.pipeline)
    tune = None
    if args.tune:
        integ.set_tune(*[int(v) for v in args.tune.split(",")])
        tune = integ.tune()
    elif not args.no_autotune:
        # untimed: pick the launch configuration on this workload (the state
        # is not modified)
        tune = integ.autotune(state, cfg["dt"], reps=2)
        if args.serialize:
            integ.set_tune(tune["cg_variant"], tune["cg_blocks"], tune["cyclic"], 1)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    state0 = None if args.no_gate else state.clone()
    for _ in range(args.warmup):
        integ.step(state, cfg["dt"])
    torch.cuda.synchronize()
    native.misdc_reset_profile(integ.handle)
    torch.cuda.synchronize()
    if args.nu_tol > 0:
        # adaptive nested iterations: the passes of every step are counted
        # (read between steps, outside the timed intervals)
        elapsed, passes = 0.0, []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            integ.step(state, cfg["dt"])
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            passes.append(integ.stats()["nested_passes"])
        stats = integ.stats()
        updates = n * M * sum(sum(p) for p in passes)
    else:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            integ.step(state, cfg["dt"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = integ.stats()          # last step's counters + timings over all timed steps
        elapsed = t1 - t0
        passes = None
        updates = n * M * cfg["nu"] * cfg["sweeps"] * args.steps
    value = updates / elapsed
    profiled_ms = elapsed / args.steps * 1e3
    newton_per_cell = stats["newton_iters"] / max(1, stats["newton_solves"])
    newton_sweeps = newton_sweep_stats(integ, cfg["sweeps"])
    cg_per_solve = stats["cg_iters"] / max(1, stats["cg_solves"])
    variant = integ.tune()["cg_variant"]
    # the eager integrator is closed before the graph leg and the gate build
    # their own: its streams would otherwise share the hardware queues with
    # theirs
    integ.close()
    # the same steps without timing events, issued eagerly and replayed as
    # graphs; the faster of the two is the measurement (fixed passes only:
    # adaptive passes read the host between passes)
    legs = {}
    if args.nu_tol <= 0:
        legs["eager"] = timed_leg(mh, g, cfg, state_init, args, tune, False)
        if not args.no_graph:
            legs["graph"] = timed_leg(mh, g, cfg, state_init, args, tune, True)
    execution = "eager_profiled"
    if legs:
        execution = min(legs, key=lambda k: legs[k]["ms_per_step"])
        value = legs[execution]["value"]
        elapsed = legs[execution]["ms_per_step"] * args.steps * 1e-3
    graph = legs.get("graph")

    # roofline of the dominant kernel
    d_ms, d_n = stats["diffusion_kernel_ms"], stats["diffusion_kernel_launches"]
    r_ms, r_n = stats["newton_kernel_ms"], stats["newton_kernel_launches"]
    if d_ms >= r_ms:
        avg_s = d_ms / max(1, d_n) * 1e-3
        unknowns = 8 * n + n            # 8 diffused species + enthalpy
        traffic = CG_BYTES_PER_UNKNOWN_ITER * unknowns * cg_per_solve
        achieved = traffic / avg_s / 1e9
        cg_names = {0: "cg_kernel (vectors in global memory)",
                    1: "cg_regs_kernel<9,1,512> (register-resident, diagonal preconditioner)",
                    2: "cg_regs_kernel<9,2,256>", 4: "cg_regs_kernel<9,4,256>",
                    101: "cg_tile_kernel<9,1> (32x16 tiles, 1 local preconditioner sweep)",
                    102: "cg_tile_kernel<9,2> (32x16 tiles, 2 local preconditioner sweeps)",
                    103: "cg_tile_kernel<9,3> (32x16 tiles, 3 local preconditioner sweeps)"}
        roof = {"kernel": cg_names.get(variant, str(variant)) + ": batched pipelined PCG, "
                          "implicit diffusion of 9 fields",
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic("pmc_cg_kernel_flame2d_256.md",
                                            "paper_1801_01201_amd/csrc/cg.hip"),
                "avg_launch_ms": avg_s * 1e3, "launches": d_n,
                "algorithmic_bytes_per_launch": traffic,
                "cg_iterations_per_launch": cg_per_solve}
    else:
        avg_s = r_ms / max(1, r_n) * 1e-3
        flops = NEWTON_FLOP_PER_ITER_9 * n * newton_per_cell
        achieved = flops / avg_s / 1e12
        roof = {"kernel": ("newton_spec (reaction solve generated for the mechanism)"
                           if native.misdc_mech_specialized(mh.handle)[0] else
                           "newton_kernel<9, true> (per-cell reaction solve, inert bath "
                           "eliminated)"), "bound": "alu",
                "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": (measured_traffic("pmc_newton_spec_flame2d_256.md",
                                             "paper_1801_01201_amd/csrc/chem_spec.cpp")
                            if native.misdc_mech_specialized(mh.handle)[0] else
                            measured_traffic("pmc_newton_kernel_flame2d_256.md",
                                             "paper_1801_01201_amd/csrc/chem.hip")),
                "avg_launch_ms": avg_s * 1e3, "launches": r_n}
    # the reaction solve's own roofline, whichever kernel dominates: FP64 work
    # against the vector peak, and its algorithmic HBM bytes against 8 TB/s
    r_avg = r_ms / max(1, r_n) * 1e-3
    spec_ok, _ = native.misdc_mech_specialized(mh.handle)
    r_flops = NEWTON_FLOP_PER_ITER_9 * n * newton_per_cell
    r_bytes = NEWTON_BYTES_PER_SOLVE_9 * n
    roof_r = None if r_n == 0 else {
        "kernel": ("newton_spec (reaction solve generated for the mechanism, one thread per "
                   "cell-node)" if spec_ok else "newton_kernel<9, true>"),
        "bound": "alu", "achieved": r_flops / r_avg / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": r_flops / r_avg / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
        "hbm_achieved_GBs": r_bytes / r_avg / 1e9, "hbm_frac": r_bytes / r_avg / 1e9 / HBM_PEAK_GBS,
        "avg_launch_ms": r_avg * 1e3, "launches": r_n,
        "algorithmic_flops_per_launch": r_flops, "algorithmic_bytes_per_launch": r_bytes,
        "traffic": (measured_traffic("pmc_newton_spec_flame2d_256.md",
                                     "paper_1801_01201_amd/csrc/chem_spec.cpp")
                    if spec_ok else None)}
    other = {"diffusion_solve_ms_per_launch": d_ms / max(1, d_n),
             "newton_ms_per_launch": r_ms / max(1, r_n),
             "diffusion_solve_share_of_step": d_ms / (profiled_ms * args.steps),
             "newton_share_of_step": r_ms / (profiled_ms * args.steps)}
    gate = None if args.no_gate else accuracy_gate(cfg, mech, mh, state0, tune)
    g.close()
    line = {
        "metric": METRIC, "value": value, "unit": "cell-node updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"flame2d_256: 2-D periodic {nx}x{ny} flame, 9 species / 21 "
                               f"reactions, CISDCQ-{cfg['nu']}"
                               + (f" (adaptive, at most {cfg['nu']} passes, nu_tol "
                                  f"{args.nu_tol})" if args.nu_tol > 0 else "")
                               + f", {cfg['n_nodes']} Gauss-Lobatto "
                               f"nodes, {cfg['sweeps']} sweeps, dt {cfg['dt']} s",
                   "cells": n, "nodes": cfg["n_nodes"], "sweeps": cfg["sweeps"],
                   "nu": cfg["nu"], "scheme": cfg["scheme"], "serialize": args.serialize,
                   "pipeline": args.pipeline,
                   "nu_tol": args.nu_tol, "cg_rtol": args.cg_rtol},
        "nested_passes_per_step": passes,
        "sweep_increment_last_step": stats["sweep_increment"],
        "newton_iters_per_cell": newton_per_cell,
        "newton_iters_per_sweep": newton_sweeps,
        "newton_pivot_retries_last_step": stats.get("newton_pivot_retries"),
        "cg_iters_per_solve": cg_per_solve,
        "cell_node_updates_per_step_incl_node0": n * (M + 1) * cfg["nu"] * cfg["sweeps"],
        "roofline": roof,
        "roofline_reaction_solve": roof_r,
        "fp64_counters": fp64_counter_rates(d_ms, d_n, r_ms, r_n, spec_ok),
        "kernel_split": other,
        "autotune": tune,
        "execution": execution,
        "eager_profiled_ms_per_step": profiled_ms,
        "eager_ms_per_step": legs["eager"]["ms_per_step"] if "eager" in legs else None,
        "graph_ms_per_step": graph["ms_per_step"] if graph else None,
        "graph_replay": graph,
        "cpu_baseline": cpu,
        "accuracy_gate": gate,
        "newton_failed": stats["newton_failed"], "cg_failed": stats["cg_failed"],
    }
    # a run with unconverged solves or a failed gate is not a measurement
    line["valid"] = bool(stats["converged"] and (gate is None or gate["passed"])
                         and all(leg["converged"] for leg in legs.values()))
    print(json.dumps(line), flush=True)
    if not line["valid"]:
        print("[bench] INVALID: unconverged solves or failed accuracy gate", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
