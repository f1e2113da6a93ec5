"""Autotuner for the particle-tile shape, workgroup size, launch options and schedule.

For a workload it builds short-lived simulations with each candidate
(tile shape, threads per workgroup), times a few steps with HIP events
(pic_profile) and keeps the fastest; with that tile it then times the launch
options (2D field-tile heights, inline or deferred particle launch) and keeps
the fastest set; for batches it also compares the batched and the
per-instance schedules.  Results are cached in a JSON file keyed by
the workload's shape so later runs reuse them.
"""
import json
import os
import time

from . import _lib as L
from .sim import Simulation

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

CANDIDATES_2D = [((16, 1, 16), 256), ((16, 1, 16), 512), ((32, 1, 16), 256), ((16, 1, 32), 256),
                 ((32, 1, 32), 512), ((8, 1, 16), 256), ((8, 1, 8), 256)]
CANDIDATES_3D = [((8, 4, 4), 256), ((8, 2, 4), 256), ((4, 4, 8), 256), ((8, 8, 4), 256), ((4, 4, 4), 256)]
# launch options tried with the chosen tile ({} = the library's defaults);
# every one leaves the results unchanged
# (the field-tile heights and particle launch forms are bitwise neutral; the
# re-sort period changes which tile deposits a particle, so FP32 results move
# within rounding)
OPTIONS_2D = [{}, {"seen_tile_z": 16, "yee_tile_z": 8}, {"seen_tile_z": 32}, {"seen_tile_z": 32, "yee_tile_z": 16},
              {"seen_tile_z": 64, "yee_tile_z": 16}, {"seen_tile_z": 128}, {"particle_defer": 0}, {"particle_defer": 1},
              {"particle_prefetch": 1}, {"particle_waves4": 1}, {"resort_every": 8}, {"resort_every": 32}]
OPTIONS_3D = [{}, {"resort_every": 8}, {"resort_every": 32}]
MARGIN = 0.01


def key(workloads, precision):
    """Cache key: dimensions, order, density, precision, scheme (gather, solver,
    correction) and the batch's size and leading grid shapes."""
    w = workloads[0]
    sizes = sorted(tuple(x["n"]) for x in workloads)
    corr = w.get("correction")
    scheme = "%s-%s-%s" % (w.get("interp", "galerkin"), w.get("solver", "yee"),
                           "ratio" if corr == "ratio" else ("psi" if corr else "none"))
    return "%dd_o%d_ppc%d_%s_%s_n%d_%s" % (w["dims"], w["order"], w["ppc"], precision, scheme, len(workloads),
                                           "-".join("x".join(map(str, s)) for s in sizes[:4]))


def lookup(workloads, precision, cache=CACHE):
    """The cached tuning of these workloads, or None; never runs the tuner."""
    if isinstance(workloads, dict):
        workloads = [workloads]
    return _load_cache(cache).get(key(workloads, precision)) if cache else None


def _load_cache(path):
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            return {}
    return {}


def apply_options(sim, options):
    """Set the launch options a tuning result chose on a Simulation."""
    for name, value in (options or {}).items():
        sim.set_option(name, value)


def tune(workloads, particles, precision="fp32", steps=10, warmup=3, cache=CACHE, candidates=None,
         options=None):
    """Return {"tile": [tx, ty, tz], "block": b, "options": {...}, "schedule": "batched"|"plain",
    "step_ms": t}; apply "options" with apply_options."""
    if isinstance(workloads, dict):
        workloads, particles = [workloads], [particles]
    k = key(workloads, precision)
    db = _load_cache(cache) if cache else {}
    if k in db:
        return db[k]
    dims = workloads[0]["dims"]
    cands = candidates or (CANDIDATES_2D if dims == 2 else CANDIDATES_3D)
    best = None
    for tile, block in cands:
        if dims == 3 and any(t > n for t, n in zip(tile, workloads[0]["n"])):
            continue
        try:
            sim = Simulation(workloads, particles, precision=precision, tile=tile, block=block)
        except L.PicError:
            continue                # e.g. a tile window that does not fit in LDS
        sim.step(warmup)
        prof = sim.profile(steps)
        sim.close()
        if best is None or prof["step_ms"] < best["step_ms"]:
            best = {"tile": list(tile), "block": block, "step_ms": prof["step_ms"]}
    best["options"] = {}
    for opts in (options if options is not None else (OPTIONS_2D if dims == 2 else OPTIONS_3D)):
        if not opts:
            continue
        if precision != "fp32" and any(k in opts for k in ("particle_prefetch", "particle_waves4")):
            continue
        sim = Simulation(workloads, particles, precision=precision, tile=best["tile"], block=best["block"])
        apply_options(sim, opts)
        sim.step(warmup)
        prof = sim.profile(steps)
        sim.close()
        # a set replaces the library's defaults only when it is clearly faster
        # (run-to-run spread of these short timings is about 1 %)
        if prof["step_ms"] < best["step_ms"] * (1.0 - MARGIN):
            best["options"], best["step_ms"] = dict(opts), prof["step_ms"]
    best["schedule"] = "batched"
    if len(workloads) > 1:
        times = {}
        for sched in ("batched", "plain"):
            sim = Simulation(workloads, particles, precision=precision, tile=best["tile"], block=best["block"])
            apply_options(sim, best["options"])
            sim.set_schedule(sched, True)
            sim.step(warmup)
            sim.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            sim.synchronize()
            times[sched] = (time.perf_counter() - t0) / steps * 1e3
            sim.close()
        best["schedule"] = min(times, key=times.get)
        best["schedule_ms"] = times
    if cache:
        db[k] = best
        with open(cache + ".tmp", "w") as f:
            json.dump(db, f, indent=1)
        os.replace(cache + ".tmp", cache)
    return best
