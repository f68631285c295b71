"""Benchmark: MG-CCCS solves of the 1025^2 Temkin-Poet problem on one MI355X.

A step is one pass of the whole hot path over one batch: the three FP64
MG-CCCS solves of the 1025^2 workload (domain [0,80]^2, ECS beyond 60 at pi/6,
7 levels, 8 channels, E = 0.05, 0.5, 2.0 solved separately) from the seeded
complex-normal initial guess to a relative residual of 1e-10.  Setup
(set_potential / set_energy) happens before the timed region; right-hand side,
initial guess and workspace are resident in HBM when it starts.

value = solved unknowns per second = 3 * 1023^2 / (seconds per step).

Further legs of the same JSON line:
  mixed          the same step with the complex-FP32 MG-CCCS cycle inside the
                 FP64 FGMRES;
  bicgstab       the same step with MG-CCCS-preconditioned BiCGSTAB instead of
                 FGMRES, FP64 and FP32 cycles;
  batched        the step's solves run together through the batch entry point,
                 FP64 and FP32 cycles;
  c2             the 2049^2 workload (E = 0.1): one FP64 and one mixed solve;
  c3             the 64-solve batch workload: mixed precision through the batch
                 entry point against plain FP64 solves one after another;
  hbm_4097       a 4097^2 grid (every FP64 field larger than the on-die cache):
                 the finest-level streaming kernels timed with HIP events,
                 algorithmic bytes / time against the 8 TB/s HBM peak;
  kernels        the same per-kernel figures on the timed 1025^2 workload;
  roofline       the dominant kernel, timed with HIP events on the library's
                 stream inside the timed steps;
  cpu_baseline   the FP64 CPU oracle on a bounded sample of the step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FGMRES restart length of every timed solve: the fastest measured at 1025^2
# and 2049^2 in both cycle precisions (6 against 4, 5, 7, 8, 10, 12)
RESTART = 6
HBM_PEAK_GBS = 8000.0                  # MI355X HBM3E, published
# kernel classes of the library's event timer, by short name
KCLASS = {"apply_dot": 1, "axpy": 2, "s1": 3, "s2": 4, "cccs_project": 5, "cccs_chain": 6,
          "s1_fine": 7, "s2_fine": 8, "cccs_expand": 9}
# the kernel whose roofline the line reports: the largest share of the step's
# kernel time among single kernels in the committed rocprofv3 summary
ROOFLINE_KERNEL = "apply_dot"
# per-kernel figures reported beside it (the finest-level streaming passes)
PROBE_KERNELS = ["s1_fine", "s2_fine", "cccs_project", "cccs_expand", "apply_dot", "axpy"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--max-it", type=int, default=20000)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-bicgstab", action="store_true", help="skip the BiCGSTAB outer-solver leg")
    p.add_argument("--no-batch", action="store_true", help="skip the batched legs")
    p.add_argument("--no-sweep", action="store_true", help="skip the cross-section sweep leg")
    p.add_argument("--no-c2", action="store_true", help="skip the 2049^2 leg")
    p.add_argument("--no-hbm", action="store_true", help="skip the 4097^2 bandwidth leg")
    p.add_argument("--no-c3", action="store_true", help="skip the 64-solve batch leg")
    p.add_argument("--no-kernels", action="store_true", help="skip the per-kernel 1025^2 figures")
    p.add_argument("--only-hbm", action="store_true", help="only the 4097^2 leg (profiling runs)")
    p.add_argument("--energies", type=str, default="0.05,0.5,2.0",
                   help="subset of the workload energies (profiling runs)")
    p.add_argument("--roofline-kernel", type=str, default=ROOFLINE_KERNEL, choices=sorted(KCLASS))
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a plain device copy of known size (counter calibration)")
    p.add_argument("--cpu-iters", type=int, default=20,
                   help="oracle FGMRES iterations timed per energy for the CPU baseline")
    return p.parse_args()


def make_problem(w, torch, fp32=True):
    """Handle with the tuned preconditioning hierarchy (autotuner cache),
    right-hand side, initial guess and solution field."""
    from paper_1412_1953_amd import autotune
    from paper_1412_1953_amd.workloads import initial_guess
    g = autotune.tuned_grid(w, max_restart=RESTART, fp32=fp32)
    chi = g.build_rhs_tp(g.field())
    u0 = g.from_numpy(initial_guess(w.n, w.seed))
    u = g.field()
    return g, chi, u0, u


def run_step(problems, inner, torch, max_it, tol=1e-10, outer=None):
    from paper_1412_1953_amd import mgcccs
    outer = mgcccs.FGMRES if outer is None else outer
    out = []
    for g, chi, u0, u in problems:
        u.copy_(u0)
        r = g.solve(u, chi, outer=outer, inner=inner, restart=RESTART, max_it=max_it, tol=tol)
        out.append(r)
    return out


def rel_diff(problems, ref):
    """Relative 2-norm difference of each handle's current solution from the
    reference solution (the FP64 FGMRES step's), over the interior nodes."""
    out = []
    for (_, _, _, u), r in zip(problems, ref):
        a, b = u[1:-1, 1:-1], r[1:-1, 1:-1]
        out.append(float((a - b).norm() / b.norm()))
    return out


def use_schedule(problems, inner, wls):
    """The tuned launch schedule of each handle for the cycle precision."""
    from paper_1412_1953_amd import autotune, mgcccs
    for (g, *_), w in zip(problems, wls):
        g.set_schedule(*autotune.schedule_of(w, inner == mgcccs.FP32))


def time_steps(problems, inner, torch, steps, warmup, max_it, kclass=0, tol=1e-10, outer=None):
    """Seconds per step; with kclass, the library's HIP-event timer brackets
    the launches of that kernel inside the timed steps (on the stream they
    run on), in every fourth restart cycle of each solve.
    The timer is selected before the warmup, so that the restart graphs with
    the event nodes are captured outside the timed region."""
    for g, *_ in problems:
        g.set_kernel_timer(kclass)
    for _ in range(warmup):
        run_step(problems, inner, torch, max_it, tol, outer)
    torch.cuda.synchronize()
    for g, *_ in problems:
        g.read_kernel_timer()                      # drop the warmup's figures
    t0 = time.perf_counter()
    res = []
    for _ in range(steps):
        res = run_step(problems, inner, torch, max_it, tol, outer)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = launches = nbytes = floor = 0
    for g, *_ in problems:
        a, b, c, d = g.read_kernel_timer()
        ms, launches, nbytes, floor = ms + a, launches + b, nbytes + c, floor + d
        g.set_kernel_timer(0)
    return dt, res, (ms, launches, nbytes, floor)


def kernel_figure(timing):
    """GB/s of one kernel class from the timer's (ms, launches, bytes, floor):
    event brackets minus the bracket of an empty launch recorded before each."""
    ms, launches, nbytes, floor = timing
    if launches <= 0:
        return None
    avg_s = (ms - floor) * 1e-3 / launches
    achieved = nbytes / launches / avg_s / 1e9
    return {"achieved_gbs": achieved, "frac_hbm": achieved / HBM_PEAK_GBS, "avg_us": avg_s * 1e6,
            "avg_us_raw_events": ms * 1e3 / launches, "event_floor_us_per_launch": floor * 1e3 / launches,
            "bytes_per_launch": nbytes / launches, "launches": launches}


def per_kernel(problems, inner, torch, max_it, kernels):
    """Per-kernel timer figures over one more run of the solves (outside the
    timed steps), one class per run."""
    out = {}
    for k in kernels:
        _, _, t = time_steps(problems, inner, torch, 1, 0, max_it, KCLASS[k])
        out[k] = kernel_figure(t)
    return out


def time_batch(problems, inner, torch, steps, warmup, max_it):
    """Seconds per step with the step's solves run together through the batch
    entry point (one graph per unfinished solve and restart round, launched
    over the batch's streams, one synchronisation per round)."""
    from paper_1412_1953_amd import mgcccs
    batch = mgcccs.Batch([g for g, *_ in problems])
    us = [p[3] for p in problems]
    fs = [p[1] for p in problems]

    def one():
        for _, _, u0, u in problems:
            u.copy_(u0)
        return batch.solve(us, fs, inner=inner, restart=RESTART, max_it=max_it, tol=1e-10)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(steps):
        res = one()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, res


def time_sweep(problem, E, torch, calls=20, npairs=256):
    """Wall-clock milliseconds per energy-sharing sweep of the ionisation
    amplitude at excess energy E (npairs momentum pairs in one
    mgc_cross_section_sweep call, the synchronising read-back included) on the
    step's converged solution."""
    from paper_1412_1953_amd import mgcccs
    g, chi, _, u = problem
    alphas = [0.01 + (math.pi / 2 - 0.02) * a / (npairs - 1) for a in range(npairs)]
    k1s, k2s = mgcccs.sharing_momenta(E, alphas)
    g.cross_section_sweep(u, chi, k1s, k2s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        zs, _ = g.cross_section_sweep(u, chi, k1s, k2s)
    dt = (time.perf_counter() - t0) / calls
    return {"pairs": npairs, "excess_energy": E, "ms_per_call": dt * 1e3,
            "zeta_max": max(abs(z) for z in zs)}


def c2_leg(torch, max_it):
    """The 2049^2 workload: one FP64 and one mixed (FP32 cycle) solve, each
    timed once after one untimed solve."""
    from paper_1412_1953_amd import mgcccs
    from paper_1412_1953_amd.workloads import TP2049 as w
    prob = make_problem(w, torch)
    out = {"workload": w.name, "n": w.n, "E": w.E, "tol": w.tol}
    ref = None
    for name, inner in (("fp64", mgcccs.FP64), ("mixed", mgcccs.FP32)):
        use_schedule([prob], inner, [w])
        dt, res, _ = time_steps([prob], inner, torch, 1, 1, max_it)
        r = res[0]
        out[name] = {"value": w.unknowns / dt, "ms": dt * 1e3, "iters": r.iters, "relres": r.relres,
                     "status": r.status}
        if ref is None:
            ref = [prob[3].clone()]
        else:
            out[name]["rel_diff_vs_fp64"] = rel_diff([prob], ref)[0]
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    del prob, ref
    torch.cuda.empty_cache()
    return out


def c3_leg(torch, max_it):
    """The 64-solve batch workload (257^2 / 513^2 / 1025^2, E in [0.02, 3.0],
    4..16 channels, each with its tuned hierarchy and schedule): all solves
    together through the batch entry point with the complex-FP32 cycle, and
    the same solves one after another with the FP64 cycle, each timed once
    after an untimed warm-up pass (graph capture)."""
    from paper_1412_1953_amd import autotune, mgcccs
    from paper_1412_1953_amd.workloads import batch_workloads, initial_guess
    wls = batch_workloads()
    t0 = time.perf_counter()
    probs = []
    for w in wls:
        g = autotune.tuned_grid(w, fp32_cycle=True, max_restart=RESTART, fp32=True)
        probs.append((g, g.build_rhs_tp(g.field()), g.from_numpy(initial_guess(w.n, w.seed)), g.field()))
    setup_s = time.perf_counter() - t0
    unknowns = sum(w.unknowns for w in wls)
    out = {"solves": len(wls), "unknowns": unknowns, "setup_s": setup_s}
    batch = mgcccs.Batch([p[0] for p in probs])
    us, fs = [p[3] for p in probs], [p[1] for p in probs]
    for timed in (False, True):
        for _, _, u0, u in probs:
            u.copy_(u0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rb = batch.solve(us, fs, inner=mgcccs.FP32, restart=RESTART, max_it=max_it, tol=1e-10)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t1
    out["batched_mixed"] = {"value": unknowns / dtb, "s": dtb, "iters": sum(r.iters for r in rb),
                            "max_relres": max(r.relres for r in rb),
                            "converged": sum(r.status == mgcccs.MGC_OK for r in rb)}
    mixed_sol = [p[3].clone() for p in probs]
    for (g, *_), w in zip(probs, wls):
        g.set_schedule(*autotune.schedule_of(w, False))
    for timed in (False, True):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rs = run_step(probs, mgcccs.FP64, torch, max_it)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t1
    out["sequential_fp64"] = {"value": unknowns / dts, "s": dts, "iters": sum(r.iters for r in rs),
                              "max_relres": max(r.relres for r in rs),
                              "converged": sum(r.status == mgcccs.MGC_OK for r in rs)}
    # the batched mixed solutions against the FP64 ones (their largest difference)
    out["batched_mixed"]["max_rel_diff_vs_fp64"] = max(
        rel_diff([(None, None, None, m) for m in mixed_sol], [p[3] for p in probs]))
    out["speedup_batched_mixed_vs_fp64"] = dts / dtb
    del batch, probs, mixed_sol
    torch.cuda.empty_cache()
    return out


def hbm_leg(torch, kernels, iters=50, ceiling=True):
    """4097^2 probe: every FP64 field (270 MB) exceeds the 256 MB on-die cache,
    so the finest-level passes stream from HBM.  Each kernel class is timed
    over a short FGMRES(RESTART) run of `iters` iterations (the library's
    timer samples every fourth restart cycle, the first included)."""
    from paper_1412_1953_amd import mgcccs
    from paper_1412_1953_amd.workloads import TP4097 as w
    t0 = time.perf_counter()
    prob = make_problem(w, torch, fp32=False)
    setup_s = time.perf_counter() - t0
    out = {"workload": w.name, "n": w.n, "field_bytes": (w.n + 1) * prob[0].pitch * 16,
           "iterations_per_run": iters, "setup_s": setup_s}
    figs = {}
    use_schedule([prob], mgcccs.FP64, [w])
    for k in kernels:
        _, res, t = time_steps([prob], mgcccs.FP64, torch, 1, 1, iters, KCLASS[k], tol=1e-300)
        figs[k] = kernel_figure(t)
    out["kernels"] = figs
    del prob
    torch.cuda.empty_cache()
    # skipped in counter runs (--copy-probe), where its copy would be taken
    # for the calibration copy
    if ceiling:
        out["stream_ceiling"] = stream_ceiling(torch, 2 * out["field_bytes"])
    return out


def stream_ceiling(torch, nbytes, reps=20):
    """What plain streaming reaches on this device, beside the 8 TB/s
    published peak: torch's device copy (read + write bytes counted) and a
    read-only sum over an nbytes buffer, each timed with events over reps."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    res = {"bytes": nbytes}
    for name, fn, moved in (("copy_gbs", lambda: dst.copy_(src), 2 * nbytes),
                            ("read_gbs", lambda: src.sum(), nbytes)):
        fn()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        t1.synchronize()
        res[name] = moved * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return res


def traffic_from_profile(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.txt")
    src = os.path.join(ROOT, "paper_1412_1953_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(src, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if fields.get("kernels.hip sha256") != sha or "traffic bytes per launch" not in fields:
        return None
    return float(fields["traffic bytes per launch"])


def profiler_duration(kclass):
    """Mean kernel duration (us) of timer class `kclass` on the timed workload
    from the committed rocprofv3 summary, or None when there is none or the
    kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "kernels_tp1025_fp64_3energies.txt")
    src = os.path.join(ROOT, "paper_1412_1953_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    with open(src, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    lines = open(path).read().splitlines()
    if f"kernels.hip sha256: {sha}" not in lines:
        return None
    for ln in lines:
        parts = ln.split()
        if len(parts) >= 4 and parts[0] == kclass and parts[1].isdigit():
            return float(parts[2])
    return None


def copy_probe(torch):
    """A plain 256 MiB device-to-device copy, the reference for the byte
    counters (read and write sizes known exactly)."""
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def host_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wls, iters_needed, sample_iters):
    """The FP64 CPU oracle on a bounded sample of the step: for each of the
    step's energies, `sample_iters` FGMRES(RESTART) iterations of the oracle (same
    grid, right-hand side, initial guess and preconditioner) are timed; the
    solve time is that rate times the iterations the solve needs (the GPU
    solve's count: the two follow the same iteration), setup excluded as on
    the GPU.  Run on one thread (twice, the faster rate of each energy kept:
    the host's other load has slowed single runs by up to 1.7x) and on every
    core of the process's affinity mask."""
    from threadpoolctl import threadpool_limits

    from oracle.solvers import MGCCCS
    from paper_1412_1953_amd import autotune
    from paper_1412_1953_amd.workloads import initial_guess
    solvers = []
    for w in wls:
        o = MGCCCS.from_workload(w, **autotune.hierarchy_of(w))
        solvers.append((w, o, o.rhs(), initial_guess(w.n, w.seed)))
    ncores = len(os.sched_getaffinity(0))
    runs = {}
    for threads, repeats in ((1, 2), (ncores, 1)):
        with threadpool_limits(limits=threads):
            per = []
            for (w, o, f, u0) in solvers:
                best = None
                for _ in range(repeats):
                    t0 = time.perf_counter()
                    r = o.solve_fgmres(u0, f, 0.0, restart=RESTART, max_it=sample_iters)
                    dt = (time.perf_counter() - t0) / r.iters
                    best = dt if best is None else min(best, dt)
                per.append(best)
            runs[threads] = (sum(p * need for p, need in zip(per, iters_needed)), per)
    unknowns = sum(w.unknowns for w in wls)
    t1, per1 = runs[1]
    tn, pern = runs[ncores]
    return {"value": unknowns / t1, "unit": "solved unknowns/s", "cores": 1, "kind": "oracle",
            "sample": (f"{sample_iters} FGMRES({RESTART}) iterations of the oracle for each energy "
                       f"{[w.E for w in wls]} of the 1025^2 workload, timed on one host thread, best of two "
                       f"runs ({', '.join(f'{1e3 * p:.0f}' for p in per1)} ms per iteration) and scaled to "
                       f"the {iters_needed} iterations the solves need to 1e-10; setup excluded"),
            "all_cores": {"value": unknowns / tn, "threads_allowed": ncores,
                          "ms_per_iteration": [1e3 * p for p in pern]},
            "host": host_model()}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the MG-CCCS hot path is measured on a single "
              "MI355X (multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1412_1953_amd import autotune, mgcccs
    from paper_1412_1953_amd.workloads import TP1025
    mgcccs.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.copy_probe:
        copy_probe(torch)
    if a.only_hbm:
        print(json.dumps({"hbm_4097": hbm_leg(torch, PROBE_KERNELS, ceiling=not a.copy_probe)}), flush=True)
        return
    wls = [TP1025[float(E)] for E in a.energies.split(",")]
    problems = [make_problem(w, torch) for w in wls]
    unknowns = sum(w.unknowns for w in wls)
    w0 = wls[0]

    kclass = KCLASS[a.roofline_kernel]
    use_schedule(problems, mgcccs.FP64, wls)
    dt64, r64, kt = time_steps(problems, mgcccs.FP64, torch, a.steps, a.warmup, a.max_it, kclass)
    line = {
        "metric": "solved unknowns/s to 1e-10 rel. residual, mixed vs FP64 MG-CCCS; HBM GB/s",
        "value": unknowns / dt64,
        "unit": "solved unknowns/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt64 * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": "tp1025_fp64_E0.05_0.5_2.0", "n": 1024, "L": 80.0, "R0": 60.0,
                   "theta": "pi/6", "levels": 7, "channels": 8, "tol": 1e-10,
                   "outer": f"FGMRES({RESTART})", "preconditioner": "MG-CCCS V(1,1)",
                   "hierarchy": [{k: (round(math.degrees(v), 6) if k != "pc_first_level" else v)
                                  for k, v in autotune.hierarchy_of(w).items()} for w in wls],
                   "schedule_fp64": [autotune.schedule_of(w, False) for w in wls],
                   "energies": [w.E for w in wls]},
        "fp64": {"iters": [r.iters for r in r64], "relres": [r.relres for r in r64],
                 "status": [r.status for r in r64],
                 "vcycles_per_s": sum(r.vcycles for r in r64) / dt64},
    }
    # the FP64 step's solutions: every other mode's error is stated against them
    ref = [p[3].clone() for p in problems]
    fig = kernel_figure(kt)
    if fig is not None:
        line["roofline"] = {"bound": "hbm", "achieved": fig["achieved_gbs"], "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": fig["achieved_gbs"] / HBM_PEAK_GBS,
                            "traffic": traffic_from_profile(a.roofline_kernel),
                            "kernel": a.roofline_kernel, "launches": fig["launches"],
                            "avg_us": fig["avg_us"], "avg_us_raw_events": fig["avg_us_raw_events"],
                            "event_floor_us_per_launch": fig["event_floor_us_per_launch"],
                            "bytes_per_launch": fig["bytes_per_launch"]}
        # the same kernel's mean duration in the committed profiler summary of
        # this step, and the fraction it gives (a cross-check of the events)
        pd = profiler_duration(a.roofline_kernel)
        line["roofline"]["profiler_avg_us"] = pd
        line["roofline"]["profiler_frac"] = (fig["bytes_per_launch"] / (pd * 1e-6) / 1e9 / HBM_PEAK_GBS
                                             if pd else None)
    if not a.no_mixed:
        use_schedule(problems, mgcccs.FP32, wls)
        dt32, r32, _ = time_steps(problems, mgcccs.FP32, torch, a.steps, a.warmup, a.max_it)
        line["mixed"] = {"value": unknowns / dt32, "ms_per_step": dt32 * 1e3,
                         "iters": [r.iters for r in r32], "relres": [r.relres for r in r32],
                         "status": [r.status for r in r32],
                         "rel_diff_vs_fp64": rel_diff(problems, ref),
                         "speedup_vs_fp64": dt64 / dt32}
    if not a.no_bicgstab:
        # the same step with MG-CCCS-preconditioned BiCGSTAB as the outer solver
        # (two cycles per iteration), FP64 and FP32 cycle
        line["bicgstab"] = {}
        for name, inner in (("fp64", mgcccs.FP64), ("mixed", mgcccs.FP32)):
            use_schedule(problems, inner, wls)
            dtb, rb, _ = time_steps(problems, inner, torch, a.steps, a.warmup, a.max_it, outer=mgcccs.BICGSTAB)
            line["bicgstab"][name] = {"value": unknowns / dtb, "ms_per_step": dtb * 1e3,
                                      "iters": [r.iters for r in rb], "relres": [r.relres for r in rb],
                                      "status": [r.status for r in rb], "rel_diff_vs_fp64": rel_diff(problems, ref),
                                      "speedup_vs_fp64_fgmres": dt64 / dtb}
    if not a.no_batch:
        for name, inner in (("batched", mgcccs.FP64), ("batched_mixed", mgcccs.FP32)):
            use_schedule(problems, inner, wls)
            dtb, rb = time_batch(problems, inner, torch, a.steps, a.warmup, a.max_it)
            line[name] = {"value": unknowns / dtb, "ms_per_step": dtb * 1e3,
                          "iters": [r.iters for r in rb], "relres": [r.relres for r in rb],
                          "status": [r.status for r in rb],
                          "rel_diff_vs_fp64": rel_diff(problems, ref),
                          "speedup_vs_fp64": dt64 / dtb}
    if not a.no_sweep:
        line["sweep"] = time_sweep(problems[0], w0.E, torch)
    if not a.no_kernels:
        use_schedule(problems, mgcccs.FP64, wls)
        line["kernels"] = per_kernel(problems, mgcccs.FP64, torch, a.max_it, PROBE_KERNELS)
    iters_needed = [r.iters for r in r64]
    del problems, ref
    torch.cuda.empty_cache()
    if not a.no_c2:
        line["c2"] = c2_leg(torch, a.max_it)
    if not a.no_c3:
        line["c3"] = c3_leg(torch, a.max_it)
    if not a.no_hbm:
        line["hbm_4097"] = hbm_leg(torch, PROBE_KERNELS, ceiling=not a.copy_probe)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wls, iters_needed, a.cpu_iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
