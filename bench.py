"""Benchmark: MG-CCCS solves of the 1025^2 Temkin-Poet problem on one MI355X.

A step is one pass of the whole hot path over one batch: the three FP64
MG-CCCS solves of the 1025^2 workload (domain [0,80]^2, ECS beyond 60 at pi/6,
7 levels, 8 channels, E = 0.05, 0.5, 2.0 solved separately) from the seeded
complex-normal initial guess to a relative residual of 1e-10.  Setup
(set_potential / set_energy) happens before the timed region; right-hand side,
initial guess and workspace are resident in HBM when it starts.

value = solved unknowns per second = 3 * 1023^2 / (seconds per step).
The same step with the complex-FP32 preconditioner inside the FP64 FGMRES is
reported as "mixed", and the same FP64 solves run together through the batch
entry point as "batched".  "roofline" covers the dominant kernel, timed with HIP
events on the library's stream inside the timed steps; "cpu_baseline" is the
FP64 CPU oracle on a bounded sample of the same workload.
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

PC_GAMMA = math.radians(5.0)
RESTART = 10
HBM_PEAK_GBS = 8000.0                  # MI355X HBM3E, published
# kernel classes of the library's event timer, by short name
KCLASS = {"apply_dot": 1, "axpy": 2, "s1": 3, "s2": 4, "cccs_project": 5, "cccs_chain": 6}
# the kernel whose roofline the line reports: the largest share of the step's
# kernel time in the committed rocprofv3 summary
ROOFLINE_KERNEL = "s1"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--max-it", type=int, default=20000)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    p.add_argument("--no-sweep", action="store_true", help="skip the cross-section sweep leg")
    p.add_argument("--energies", type=str, default="0.05,0.5,2.0",
                   help="subset of the workload energies (profiling runs)")
    p.add_argument("--roofline-kernel", type=str, default=ROOFLINE_KERNEL, choices=sorted(KCLASS))
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a plain device copy of known size (counter calibration)")
    return p.parse_args()


def make_problem(w, torch):
    from paper_1412_1953_amd import mgcccs
    from paper_1412_1953_amd.workloads import initial_guess
    g = mgcccs.Grid.from_workload(w, pc_gamma=PC_GAMMA, max_restart=RESTART, fp32=True)
    g.set_potential(w.Z1, w.Z2, w.lam)
    g.set_energy(w.E)
    chi = g.build_rhs_tp(g.field())
    u0 = g.from_numpy(initial_guess(w.n, w.seed))
    u = g.field()
    return g, chi, u0, u


def run_step(problems, inner, torch, max_it):
    from paper_1412_1953_amd import mgcccs
    out = []
    for g, chi, u0, u in problems:
        u.copy_(u0)
        r = g.solve(u, chi, outer=mgcccs.FGMRES, inner=inner, restart=RESTART, max_it=max_it,
                    tol=1e-10)
        out.append(r)
    return out


def time_steps(problems, inner, torch, steps, warmup, max_it, kclass=0):
    """Seconds per step; with kclass, the library's HIP-event timer brackets
    every launch of that kernel inside the timed steps (on its own stream).
    The timer is selected before the warmup, so that the restart graphs with
    the event nodes are captured outside the timed region."""
    for g, *_ in problems:
        g.set_kernel_timer(kclass)
    for _ in range(warmup):
        run_step(problems, inner, torch, max_it)
    torch.cuda.synchronize()
    for g, *_ in problems:
        g.read_kernel_timer()                      # drop the warmup's figures
    t0 = time.perf_counter()
    res = []
    for _ in range(steps):
        res = run_step(problems, inner, torch, max_it)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = launches = nbytes = floor = 0
    for g, *_ in problems:
        a, b, c, d = g.read_kernel_timer()
        ms, launches, nbytes, floor = ms + a, launches + b, nbytes + c, floor + d
        g.set_kernel_timer(0)
    return dt, res, (ms, launches, nbytes, floor)


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
    mgc_cross_section_sweep call, host test functions and the synchronising
    read-back included) on the step's converged solution."""
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


def copy_probe(torch):
    """A plain 256 MiB device-to-device copy, the reference for the byte
    counters (read and write sizes known exactly)."""
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def cpu_baseline(w):
    """The FP64 CPU oracle on a bounded sample of the workload: the complete
    solve of its first energy (same grid, right-hand side, initial guess,
    FGMRES(10) with the MG-CCCS preconditioner, tolerance 1e-10) on one
    thread; setup (bound states, factorisations) excluded as on the GPU."""
    from oracle.solvers import MGCCCS
    from paper_1412_1953_amd.workloads import initial_guess
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    o = MGCCCS.from_workload(w, pc_gamma=PC_GAMMA)
    f = o.rhs()
    u0 = initial_guess(w.n, w.seed)
    t0 = time.perf_counter()
    r = o.solve_fgmres(u0, f, w.tol, restart=RESTART, max_it=20000)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister()
    return {"value": w.unknowns / dt, "unit": "solved unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"complete E={w.E} solve of the 1025^2 workload, {r.iters} FGMRES({RESTART}) "
                      f"iterations to relres {r.relres:.2e} in {dt:.1f} s on one host thread"}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the MG-CCCS hot path is measured on a single "
              "MI355X (multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1412_1953_amd import mgcccs
    from paper_1412_1953_amd.workloads import TP1025
    mgcccs.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wls = [TP1025[float(E)] for E in a.energies.split(",")]
    problems = [make_problem(w, torch) for w in wls]
    unknowns = sum(w.unknowns for w in wls)

    if a.copy_probe:
        copy_probe(torch)
    kclass = KCLASS[a.roofline_kernel]
    dt64, r64, (kms, kl, kb, kfloor) = time_steps(problems, mgcccs.FP64, torch, a.steps, a.warmup,
                                                  a.max_it, kclass)
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
                   "pc_gamma_deg": 5.0, "energies": [w.E for w in wls]},
        "fp64": {"iters": [r.iters for r in r64], "relres": [r.relres for r in r64],
                 "status": [r.status for r in r64],
                 "vcycles_per_s": sum(r.vcycles for r in r64) / dt64},
    }
    if kl > 0:
        # event brackets minus the bracket of an empty launch recorded before each
        avg_s = (kms - kfloor) * 1e-3 / kl
        achieved = kb / kl / avg_s / 1e9
        traffic = traffic_from_profile(a.roofline_kernel)
        line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                            "kernel": a.roofline_kernel, "launches": kl,
                            "avg_us": avg_s * 1e6, "avg_us_raw_events": kms * 1e3 / kl,
                            "event_floor_us_per_launch": kfloor * 1e3 / kl,
                            "bytes_per_launch": kb / kl}
    if not a.no_mixed:
        dt32, r32, _ = time_steps(problems, mgcccs.FP32, torch, a.steps, a.warmup, a.max_it)
        line["mixed"] = {"value": unknowns / dt32, "ms_per_step": dt32 * 1e3,
                         "iters": [r.iters for r in r32], "relres": [r.relres for r in r32],
                         "status": [r.status for r in r32],
                         "speedup_vs_fp64": dt64 / dt32}
    if not a.no_sweep:
        line["sweep"] = time_sweep(problems[0], wls[0].E, torch)
    if not a.no_batch:
        dtb, rb = time_batch(problems, mgcccs.FP64, torch, a.steps, a.warmup, a.max_it)
        line["batched"] = {"value": unknowns / dtb, "ms_per_step": dtb * 1e3,
                           "iters": [r.iters for r in rb], "relres": [r.relres for r in rb],
                           "status": [r.status for r in rb],
                           "speedup_vs_fp64": dt64 / dtb}
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wls[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
