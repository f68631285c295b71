"""Project autotuner of the MG-CCCS solver (runs on the GPU; the choices are
stored in ``tuning_cache.json`` next to this file and looked up by the
workload helpers).

Two kinds of choice are made by measurement, per problem:

* the preconditioning hierarchy -- on which contour each multigrid level
  smooths (Sec. 3.1: the real interior rotated by an angle; level 0 may stay
  on the exterior-complex-scaled operator itself) -- which changes how many
  FGMRES iterations a solve needs.  Keyed by grid size, domain, channel count
  and energy; chosen by complete solves from the workload's seeded guess,
  fastest converged solve wins (a candidate is stopped once it has used
  twice the iterations of the best one so far).
* the launch schedule of the cycle (``mgc_schedule``: large or small tiles
  per level, paired levels, coarse tail), which never changes the arithmetic.
  Keyed by grid size, domain, channel count and cycle precision; chosen by
  timing a fixed number of FGMRES iterations.

    python -m paper_1412_1953_amd.autotune OUT.json [workload-set ...]

tunes the named workload sets (c0, c1, c2, c3, c4; default all) and writes
the merged cache to OUT.json.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_PATH = os.path.join(_HERE, "tuning_cache.json")

# hierarchy candidates: (first rotated level, angle below it, angle from it on), degrees
HIERARCHIES = [(1, 0.0, 15.0), (1, 5.0, 15.0), (1, 10.0, 15.0), (0, 0.0, 10.0), (0, 0.0, 15.0)]
SCHEDULE_ITERS = 30
SCHEDULE_REPEATS = 3
# FGMRES restart length of the tuning solves (the timed solves use the same)
RESTART = 6

_cache = None


def hierarchy_key(w) -> str:
    return f"n={w.n} L={w.L:g} R0={w.R0:g} M={w.M} E={w.E:.6f}"


def schedule_key(w, fp32: bool) -> str:
    return f"n={w.n} L={w.L:g} R0={w.R0:g} M={w.M} {'fp32' if fp32 else 'fp64'}"


def load_cache(path: str = CACHE_PATH) -> dict:
    global _cache
    if _cache is None or path != CACHE_PATH:
        data = {"hierarchy": {}, "schedule": {}}
        if os.path.exists(path):
            with open(path) as fh:
                data = json.load(fh)
        if path != CACHE_PATH:
            return data
        _cache = data
    return _cache


def hierarchy_of(w) -> dict:
    """Preconditioning hierarchy of workload w: the tuned entry if there is
    one, else the workload's own defaults.  Keys: pc_first_level, pc_gamma0,
    pc_gamma (radians)."""
    e = load_cache()["hierarchy"].get(hierarchy_key(w))
    if e is None:
        return {"pc_first_level": w.pc_first_level, "pc_gamma0": w.pc_gamma0, "pc_gamma": w.pc_gamma}
    return {"pc_first_level": e["first"], "pc_gamma0": math.radians(e["gamma0_deg"]),
            "pc_gamma": math.radians(e["gamma_deg"])}


def schedule_of(w, fp32: bool):
    """(small_tiles, level_pairs, coarse_tail) of workload w for the FP32 or
    FP64 cycle: the tuned entry, else the library's default."""
    e = load_cache()["schedule"].get(schedule_key(w, fp32))
    return tuple(e["schedule"]) if e else (-1, 1, 1)


def tuned_grid(w, fp32_cycle: bool = False, **kw):
    """A handle for workload w with its tuned hierarchy and schedule, with
    potential and energy set."""
    from . import mgcccs
    for k, v in hierarchy_of(w).items():
        kw.setdefault(k, v)
    g = mgcccs.Grid.from_workload(w, **kw)
    g.set_schedule(*schedule_of(w, fp32_cycle))
    g.set_potential(w.Z1, w.Z2, w.lam)
    g.set_energy(w.E)
    return g


# ---------------------------------------------------------------------------
# tuning (GPU)
def _solve_time(g, w, chi, inner, max_it, tol=None):
    import torch
    from . import mgcccs
    from .workloads import initial_guess
    u = g.from_numpy(initial_guess(w.n, w.seed))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = g.solve(u, chi, outer=mgcccs.FGMRES, inner=inner, restart=RESTART, max_it=max_it,
                tol=w.tol if tol is None else tol)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def tune_hierarchy(w, max_it=4000, log=print) -> dict:
    from . import mgcccs
    best = None
    trials = []
    for first, g0, g1 in HIERARCHIES:
        cap = max_it if best is None else min(max_it, 2 * best["iters"] + 20)
        g = mgcccs.Grid.from_workload(w, pc_first_level=first, pc_gamma0=math.radians(g0),
                                      pc_gamma=math.radians(g1), max_restart=10, fp32=False)
        g.set_potential(w.Z1, w.Z2, w.lam)
        g.set_energy(w.E)
        chi = g.build_rhs_tp(g.field())
        _solve_time(g, w, chi, mgcccs.FP64, 10, tol=1e-300)          # capture + warm
        dt, r = _solve_time(g, w, chi, mgcccs.FP64, cap)
        ok = r.status == mgcccs.MGC_OK
        trials.append({"first": first, "gamma0_deg": g0, "gamma_deg": g1, "iters": r.iters, "ms": dt * 1e3,
                       "converged": ok})
        if ok and (best is None or dt < best["ms"] * 1e-3):
            best = {"first": first, "gamma0_deg": g0, "gamma_deg": g1, "iters": r.iters, "ms": dt * 1e3}
        del g
    if best is None:
        raise RuntimeError(f"no hierarchy candidate converged for {w.name}")
    best["trials"] = trials
    log(f"[tune] {w.name}: hierarchy first={best['first']} gamma0={best['gamma0_deg']} "
        f"gamma={best['gamma_deg']} ({best['iters']} it, {best['ms']:.1f} ms)")
    return best


def schedule_candidates(levels: int):
    full = (1 << levels) - 1
    out = [(-1, 1, 1)]
    for large in range(0, min(levels - 1, 4)):
        mask = full & ~((1 << large) - 1)            # the `large` finest levels on large tiles
        for pairs in (1, 0):
            for tail in (1, 0):
                out.append((mask, pairs, tail))
    return out


def tune_schedule(w, fp32: bool, hier: dict, log=print) -> dict:
    from . import mgcccs
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    g = mgcccs.Grid.from_workload(w, max_restart=10, fp32=True, **hier)
    g.set_potential(w.Z1, w.Z2, w.lam)
    g.set_energy(w.E)
    chi = g.build_rhs_tp(g.field())
    rows = []
    for sch in schedule_candidates(w.levels):
        g.set_schedule(*sch)
        _solve_time(g, w, chi, inner, SCHEDULE_ITERS, tol=1e-300)     # capture + warm
        ts = [_solve_time(g, w, chi, inner, SCHEDULE_ITERS, tol=1e-300)[0] for _ in range(SCHEDULE_REPEATS)]
        rows.append((min(ts), sch))
    rows.sort()
    best = {"schedule": list(rows[0][1]), "ms_per_iter": rows[0][0] * 1e3 / SCHEDULE_ITERS,
            "default_ms_per_iter": [r[0] for r in rows if r[1] == (-1, 1, 1)][0] * 1e3 / SCHEDULE_ITERS}
    log(f"[tune] {schedule_key(w, fp32)}: schedule {best['schedule']} {best['ms_per_iter']:.4f} ms/it "
        f"(default {best['default_ms_per_iter']:.4f})")
    return best


def workload_sets():
    from .workloads import SMALL_129, TP1025, TP1025_GRAD, TP2049, batch_workloads
    return {"c0": [SMALL_129], "c1": list(TP1025.values()), "c2": [TP2049], "c3": batch_workloads(),
            "c4": [TP1025_GRAD]}


def tune(out_path: str, sets=None, log=print) -> dict:
    data = load_cache()
    data = {"hierarchy": dict(data["hierarchy"]), "schedule": dict(data["schedule"])}
    allsets = workload_sets()
    for name in (sets or list(allsets)):
        for w in allsets[name]:
            hk = hierarchy_key(w)
            if hk not in data["hierarchy"]:
                data["hierarchy"][hk] = tune_hierarchy(w, log=log)
                with open(out_path, "w") as fh:
                    json.dump(data, fh, indent=1, sort_keys=True)
            e = data["hierarchy"][hk]
            hier = {"pc_first_level": e["first"], "pc_gamma0": math.radians(e["gamma0_deg"]),
                    "pc_gamma": math.radians(e["gamma_deg"])}
            for fp32 in (False, True):
                sk = schedule_key(w, fp32)
                if sk not in data["schedule"]:
                    data["schedule"][sk] = tune_schedule(w, fp32, hier, log=log)
                    with open(out_path, "w") as fh:
                        json.dump(data, fh, indent=1, sort_keys=True)
    with open(out_path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    return data


if __name__ == "__main__":
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    tune(sys.argv[1], sys.argv[2:] or None, log=lambda m: print(m, flush=True))
