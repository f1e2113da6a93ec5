"""Benchmark of the GPU PIC step on one MI355X.

Headline workload (the metric's own configuration): 64 independent 2D
instances of uneven size stepped together, FP32.  nx, nz are drawn from
{64, 128, 256, 512}, c dt / dz uniform in [0.3, 0.7], gamma from {10, 50, 130},
8 particles per cell (31.2 M macro-particles over 3.9 M cells), linear Galerkin
shapes, correction stencils (Psi_E / Psi_B quartics) plus a 4-pass (1,2,1)
filter per axis; cold beams along z with 1e-6 relative momentum spread.
Synthetic seeded input (pic_inputs).

A step is the whole hot path for every instance: Yee update, fields as seen by
the particles (correction + filter), gather, Boris push, move, Esirkepov
deposit, and the periodic tile re-sort check.  `value` = particle-steps per
second of the batched schedule (one launch per kernel over all instances,
HIP-graph replay) over the timed steps, inputs resident in HBM.  Next to it:
the plain schedule (one launch per instance and kernel) eager and
graph-replayed, the adjoint cost ratio, the roofline of the dominant kernel and
of the whole step, and the FP64 oracle on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extra]
Prints one JSON line (the secondary workloads with --extra).
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1401_0838_amd", "csrc", "pic_kernels.hip")
METRIC = "particle-steps/s (gather+Boris+Esirkepov) plain vs batched; adjoint cost ratio"


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def particle_kernel_bytes(n_particles, n_cells, word=4, state_bytes=24):
    """Algorithmic HBM bytes of one particle-kernel launch: every particle's state read
    and written once (state_bytes each way), the six seen-field components read once
    and the three current components written once per cell."""
    return 2 * state_bytes * n_particles + 9 * word * n_cells


def step_bytes(n_particles, n_cells, word=4, state_bytes=24):
    """Algorithmic HBM bytes of one whole step: the particle state read and written
    once, and 24 words per cell (the Yee update reads E, B, J and writes E, B; the
    gather reads the six seen components; the deposit writes J)."""
    return 2 * state_bytes * n_particles + 24 * word * n_cells


def stored_traffic(name):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel source; else None.  Returns (bytes, source file)."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None, None
    doc = json.load(open(path))
    if doc.get("kernel_source_sha") != kernel_sha():
        return None, None
    return doc.get("hbm_bytes_per_launch"), "profiles/" + name


VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock (no packed FP32)


def valu_issue(case, n_part, launch_ms):
    """Fraction of the vector-ALU issue ceiling a particle-kernel launch reaches:
    lane instructions per particle from committed SQ_INSTS_VALU counter runs
    (only if they were taken on the current kernel source) times the particles,
    over the measured launch duration."""
    name = "valu_k_particles.json"
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    if doc.get("kernel_source_sha") != kernel_sha() or case not in doc.get("cases", {}):
        return None
    per = doc["cases"][case]["valu_lane_instr_per_particle"]
    achieved = per * n_part / (launch_ms * 1e-3)
    return {"bound": "alu", "valu_lane_instr_per_particle": per, "achieved": achieved / 1e12,
            "peak": VALU_PEAK_LANE_INSTR / 1e12, "unit": "T lane-instr/s", "frac": achieved / VALU_PEAK_LANE_INSTR,
            "source": "profiles/" + name}


# ------------------------------------------------------------------ batch

def batch_instances(accept):
    """The 64-instance batch: the first 64 candidates whose correction `accept`
    (the library's or the oracle's coefficient check) takes."""
    import pic_inputs as pi
    out = []
    for cand in pi.batched_candidates(0):
        if accept(cand):
            out.append(cand)
        if len(out) == 64:
            break
    return out


def _oracle_accepts(cand):
    from oracle import psi as opsi
    a, b, _ = opsi.psi_coeffs("galerkin", cand["alpha"])
    return opsi.psi_positive(a, b)


# ---------------------------------------------------------- CPU baseline

def _oracle_job(args):
    wl, steps = args
    import pic_inputs as pi
    from oracle.ref import OracleSim
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], wl["seeds"][0])
    sim = OracleSim(wl, x, u)
    t0 = time.perf_counter()
    sim.step(steps)
    return x.shape[0] * steps, time.perf_counter() - t0


def cpu_baseline(target_s=12.0):
    """The FP64 C oracle as it stands, on a bounded sample of the batch: one
    instance per process, each stepped serially.  Leg 1: one thread, the batch's
    first instances in order until about target_s seconds of work.  Leg 2: one
    process per host core (at most 16, the host share of one GPU), the first
    `cores` instances each for the same number of steps.  Runs before anything
    touches the GPU."""
    insts = batch_instances(_oracle_accepts)
    rate_1 = 1.6e6                                   # particle-steps/s, for sizing the sample
    steps = 4
    sample, work = [], 0
    for w in insts:
        n = w["ppc"] * w["n"][0] * w["n"][1]
        if sample and (work + n * steps) / rate_1 > target_s:
            break
        sample.append(w)
        work += n * steps
    t0 = time.perf_counter()
    ps1 = sum(_oracle_job((w, steps))[0] for w in sample)
    t1 = time.perf_counter() - t0
    cores = max(1, min(16, os.cpu_count() or 1))
    jobs = [(w, steps) for w in insts[:cores]]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_job, jobs)
    tn = time.perf_counter() - t0
    psn = sum(r[0] for r in res)
    return {"value": ps1 / t1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the batch's first %d instances (%d particles), FP64 C oracle, one thread, %.1f s"
                      % (steps, len(sample), sum(w["ppc"] * w["n"][0] * w["n"][1] for w in sample), t1),
            "nproc": {"value": psn / tn, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
                      "sample": "%d steps of each of the batch's first %d instances, one process per instance, %.1f s"
                                % (steps, len(jobs), tn)}}


# ------------------------------------------------------------ GPU blocks

# Clock state: building a batch keeps the GPU idle for about a second of host
# work, and its clocks then ramp back up over the first tens of milliseconds of
# load: the particle kernel runs ~15 % slower for the first ~30 steps of a fresh
# run (seen on every fresh batch, whatever ran before the host setup; a preheat
# of dense matrix products removes most of it, 40 steps of the batch all of
# it).  The per-kernel profile is therefore measured on a second batch right
# before the timed steps, which puts the short timed sample in the sustained
# state that a long run (the workload's 1000 steps) spends nearly all its time in.


def timed(sim, steps):
    sim.prepare(steps)          # graphs captured before the clock starts
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    return time.perf_counter() - t0


def batched_headline(steps, warmup, profile_steps):
    import pic_inputs as pi
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd.sim import Simulation
    wls = batch_instances(lambda c: L.pic_psi_coeffs(L.PIC_GALERKIN, c["alpha"], 4)[0] == L.PIC_OK)
    parts = [pi.load_beam(2, w["n"], w["ppc"], w["gamma"], w["sigma"], w["seeds"][0]) for w in wls]
    n_part = sum(p[0].shape[0] for p in parts)
    n_cells = sum(w["n"][0] * w["n"][1] for w in wls)
    out = {"instances": len(wls), "particles": n_part, "cells": n_cells}
    # the plain schedules first (same steps), so that the batched run is timed on a
    # GPU whose clocks have left their idle state
    for graph in (False, True):
        sim = Simulation(wls, parts, precision="fp32", tuned=True)
        sim.set_schedule("plain", graph)
        sim.step(warmup)
        out["plain_%s_s" % ("graph" if graph else "eager")] = timed(sim, steps)
        sim.close()
    sim = Simulation(wls, parts, precision="fp32", tuned=True)
    sim.set_schedule("batched", True)
    out["tuning"] = sim.tuning
    sim.prepare(warmup)
    # per-kernel durations (HIP events, eager steps) on a second, identical batch,
    # measured right before the timed run: its 2 x profile_steps steps also bring
    # the GPU's clocks from the idle of the host setup to their sustained state
    # (see clock_preheat), so the timed sample is not the ramp
    ps = Simulation(wls, parts, precision="fp32", tuned=True)
    ps.set_schedule("batched", True)
    ps.step(profile_steps)
    prof = ps.profile(profile_steps)
    ps.close()
    out["kernels_ms"] = {k: prof[k] for k in ("yee_ms", "seen_ms", "particle_ms", "resort_ms", "step_ms")}
    sim.step(warmup)
    dt = timed(sim, steps)
    out["batched_s"] = dt
    d = [sim.diag(i) for i in range(len(wls))]
    out["gauss_linf_rel_max"] = max(x["gauss_linf"] / max(x["rho_max"], 1e-300) for x in d)
    out["diag_rc"] = sorted({x["rc"] for x in d})
    sim.close()
    return out


def batched_steps_only(steps, warmup):
    """The headline workload's batched graph-replayed steps alone (for counter runs)."""
    import pic_inputs as pi
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd.sim import Simulation
    wls = batch_instances(lambda c: L.pic_psi_coeffs(L.PIC_GALERKIN, c["alpha"], 4)[0] == L.PIC_OK)
    parts = [pi.load_beam(2, w["n"], w["ppc"], w["gamma"], w["sigma"], w["seeds"][0]) for w in wls]
    n_part = sum(p[0].shape[0] for p in parts)
    sim = Simulation(wls, parts, precision="fp32", tuned=True)
    sim.set_schedule("batched", True)
    sim.step(warmup)
    dt = timed(sim, steps)
    sim.close()
    return {"particles": n_part, "steps": steps, "ms_per_step": 1e3 * dt / steps}


def adjoint_block():
    """256x256, 8 ppc, 200 steps, checkpoints every 20 (FP32): backward (recompute +
    reverse sweep) time over the plain forward time, both timed after a warm-up
    that captures their graphs."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    wl = pi.workload("beam2d_256_adjoint")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    n, k = wl["steps"], wl["checkpoint"]
    fwd = Simulation(wl, (x, u), precision="fp32", tuned=True)
    fwd.step(5)
    t_step = timed(fwd, n)
    fwd.close()
    sim = Simulation(wl, (x, u), precision="fp32", adjoint_steps=n, adjoint_ckpt=k, tuned=True)
    tuning = sim.tuning
    sim.adjoint_forward(k)
    sim.adjoint_backward()
    sim.synchronize()
    t0 = time.perf_counter()
    sim.adjoint_forward(n)
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.adjoint_backward()
    t_b = time.perf_counter() - t0
    sim.close()
    return {"steps": n, "checkpoint_every": k, "forward_s": t_step, "forward_with_checkpoints_s": t_f,
            "backward_s": t_b, "ratio": t_b / t_step, "tuning": tuning}


def single_block(wl, steps, warmup, word=4, state_bytes=24, precision="fp32"):
    """One instance, batched graph replay: particle-steps/s, per-kernel times and the
    particle kernel's HBM fraction."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    x, u = pi.load_beam(wl["dims"], wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    sim = Simulation(wl, (x, u), precision=precision, tuned=True)
    tuning = sim.tuning
    n_part = x.shape[0]
    n_cells = 1
    for v in wl["n"]:
        n_cells *= v
    del x, u
    sim.step(warmup)
    dt = timed(sim, steps)
    prof = sim.profile(5)
    sim.close()
    pk = particle_kernel_bytes(n_part, n_cells, word, state_bytes)
    return {"particles": n_part, "particle_steps_per_s": n_part * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "grid_cell_updates_per_s": n_cells * steps / dt,
            "kernels_ms": {k: round(prof[k], 5) for k in ("yee_ms", "seen_ms", "particle_ms")},
            "particle_kernel_hbm_frac": pk / (prof["particle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "tuning": tuning}


def extra_blocks():
    """Secondary workloads: the 512x512 x 16 ppc case (FP32, FP64, the Uniform and
    momentum-conserving gathers, the exact ratio, CK at alpha 0.9), the 3D cubic
    case and the Sec. 3 CK setting."""
    import pic_inputs as pi
    out = {"beam2d_512_fp32": single_block(pi.workload("beam2d_512", alpha=0.5), 100, 10),
           "beam2d_512_fp64": single_block(pi.workload("beam2d_512", alpha=0.5, precision="fp64"), 50, 5, 8, 44,
                                           "fp64"),
           "beam3d_128x128x256_cubic": single_block(pi.workload("beam3d_128x128x256"), 10, 3, 4, 28)}
    for interp, corr in (("uniform", True), ("momentum", True), ("galerkin", "ratio")):
        key = interp if corr is True else "exact_ratio"
        out["beam2d_512_" + key] = single_block(pi.workload("beam2d_512", alpha=0.5, interp=interp,
                                                            correction=corr), 100, 10)
    out["beam2d_512_ck_alpha0.9"] = single_block(pi.workload("beam2d_512", alpha=0.9, solver="ck"), 100, 10)
    out["beam2d_128_ck_cubic_eq6"] = single_block(pi.workload("beam2d_128_ck"), 100, 10)
    out["gamma_scan"] = gamma_scan_block(2000)
    out["variants"] = variants_block(2000)
    return out


def gamma_scan_block(steps):
    """Sec. 3 growth-rate scan through the batched engine: the 128x128 x 16 ppc
    cubic CK setting with the Eq. 6 filter, gamma in {3, 10, 30, 130} x alpha in
    {0.3 .. 0.99}, with and without the correction, FP32, `steps` steps per batch:
    throughput, each gamma's peak growth rate and the fitted power of gamma."""
    import pic_inputs as pi
    from paper_1401_0838_amd import scan
    alphas = [0.3, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99]
    gammas = [3.0, 10.0, 30.0, 130.0]
    out = {"steps": steps, "alphas": alphas, "gammas": gammas}
    for corr in (True, False):
        base = pi.workload("beam2d_128_ck", correction=corr)
        pts, wls, parts, skipped = scan.scan_instances(base, alphas, gammas)
        n_part = sum(p[0].shape[0] for p in parts)
        info = {}
        t0 = time.perf_counter()
        traces, wkin = scan.run_scan(pts, wls, parts, steps, "fp32", info)
        dt = time.perf_counter() - t0
        rates, peaks, power = scan.growth_table(pts, traces, wkin)
        out["corrected" if corr else "uncorrected"] = {
            "instances": len(pts), "skipped": skipped, "particle_steps_per_s": n_part * steps / dt,
            "peak_growth": {"%g" % g: {"rate": v[0], "alpha": v[1]} for g, v in sorted(peaks.items())},
            "peak_power_of_gamma": power, "tuning": info["tuning"][0]}
    return out


def variants_block(steps):
    """Sec. 3's variants of its setting (and Sec. 4's one-pass-each filter): growth
    rate of each over the baseline's at gamma = 130, alpha 0.5 .. 0.99."""
    import pic_inputs as pi
    from paper_1401_0838_amd import scan
    alphas = [0.5, 0.7, 0.9, 0.99]
    info = {}
    rates, skipped = scan.variant_sweep(pi.workload("beam2d_128_ck"), alphas, 130.0, steps, info=info)
    base = rates["baseline"]
    return {"steps": steps, "alphas": alphas, "gamma": 130.0, "skipped": skipped, "tuning": info["tuning"],
            "over_baseline": {k: [None if (x is None or y in (None, 0)) else x / y for x, y in zip(v, base)]
                              for k, v in rates.items() if k != "baseline"}}


def pi_workload(name, **kw):
    import pic_inputs as pi
    return pi.workload(name, **kw)


def tune_configs():
    """Run the autotuner (tune.py) on every workload this bench times and store its
    picks in the package's tune cache, which the timed blocks then read."""
    import pic_inputs as pi
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd import scan, tune
    if os.path.exists(tune.CACHE):
        os.remove(tune.CACHE)

    def beam(wl, seed=0):
        return pi.load_beam(wl["dims"], wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], seed)

    def jobs():
        wls = batch_instances(lambda c: L.pic_psi_coeffs(L.PIC_GALERKIN, c["alpha"], 4)[0] == L.PIC_OK)
        yield "batched64_uneven_2d_ppc8_fp32", wls, [beam(w, w["seeds"][0]) for w in wls], "fp32"
        wl = pi.workload("beam2d_256_adjoint")
        yield "beam2d_256_adjoint", [wl], [beam(wl)], "fp32"
        singles = [("beam2d_512_fp32", pi.workload("beam2d_512", alpha=0.5), "fp32"),
                   ("beam2d_512_fp64", pi.workload("beam2d_512", alpha=0.5, precision="fp64"), "fp64"),
                   ("beam3d_128x128x256_cubic", pi.workload("beam3d_128x128x256"), "fp32"),
                   ("beam2d_512_uniform", pi.workload("beam2d_512", alpha=0.5, interp="uniform"), "fp32"),
                   ("beam2d_512_momentum", pi.workload("beam2d_512", alpha=0.5, interp="momentum"), "fp32"),
                   ("beam2d_512_exact_ratio", pi.workload("beam2d_512", alpha=0.5, correction="ratio"), "fp32"),
                   ("beam2d_512_ck_alpha0.9", pi.workload("beam2d_512", alpha=0.9, solver="ck"), "fp32"),
                   ("beam2d_128_ck_cubic_eq6", pi.workload("beam2d_128_ck"), "fp32")]
        for name, wl, prec in singles:
            yield name, [wl], [beam(wl)], prec
        for corr in (True, False):
            pts, wls, parts, _ = scan.scan_instances(pi.workload("beam2d_128_ck", correction=corr),
                                                     [0.3, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99],
                                                     [3.0, 10.0, 30.0, 130.0])
            yield "gamma_scan_%s" % ("corrected" if corr else "uncorrected"), wls, parts, "fp32"
        for i, (pts, wls, parts, tags, _) in enumerate(scan.variant_batches(pi.workload("beam2d_128_ck"),
                                                                              [0.5, 0.7, 0.9, 0.99], 130.0)):
            yield "variants_%d" % i, wls, parts, "fp32"

    for name, wls, parts, prec in jobs():
        t0 = time.perf_counter()
        best = tune.tune(wls, parts, precision=prec, steps=20, warmup=30)
        print(json.dumps({"tuned": name, "key": tune.key(wls, prec), "pick": best,
                          "seconds": round(time.perf_counter() - t0, 1)}), flush=True)


def copy_calibration(gib=1.0, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM counters
    (FETCH_SIZE / WRITE_SIZE) of a profiler run into bytes."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_each_way": 4 * n, "reps": reps, "GBps_read_plus_write": 8 * n / dt / 1e9}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost ratio")
    ap.add_argument("--extra", action="store_true", help="also time the secondary workloads")
    ap.add_argument("--tune", action="store_true",
                    help="only run the autotuner on every timed workload and rewrite its cache")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--only", choices=("batched", "adjoint", "extra", "cpu", "step", "cubic3d"),
                    help="run one block alone and print its JSON (for profiling); 'step' runs only "
                         "the batched graph-replayed steps of the headline workload, 'cubic3d' the "
                         "128x128x256 cubic 3D beam")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(batches would shard by instance; one large domain along z in slabs, with guard-layer "
              "exchange of E, B and J and particle migration across slab faces)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.tune:
        tune_configs()
        return
    if args.only:
        blk = {"batched": lambda: batched_headline(args.steps, args.warmup, args.profile_steps),
               "adjoint": adjoint_block, "extra": extra_blocks, "cpu": cpu_baseline,
               "step": lambda: batched_steps_only(args.steps, args.warmup),
               "cubic3d": lambda: single_block(pi_workload("beam3d_128x128x256"), args.steps, args.warmup, 4,
                                               28)}[args.only]()
        print(json.dumps({args.only: blk}), flush=True)
        return

    # the oracle first: its worker processes must not be forked from a process
    # that has initialised the GPU
    cpu = None if args.no_cpu else cpu_baseline()

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    adj = None if args.no_adjoint else adjoint_block()
    b = batched_headline(args.steps, args.warmup, args.profile_steps)
    n_part, n_cells, K = b["particles"], b["cells"], args.steps
    value = n_part * K / b["batched_s"]
    ms_step = 1e3 * b["batched_s"] / K
    pk_ms = b["kernels_ms"]["particle_ms"]
    pk_bytes = particle_kernel_bytes(n_part, n_cells)
    achieved = pk_bytes / (pk_ms * 1e-3) / 1e9
    traffic, traffic_src = stored_traffic("traffic_k_particles_batched64_fp32.json")
    sb = step_bytes(n_part, n_cells)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched64_uneven_2d_ppc8_fp32", "instances": b["instances"], "cells": n_cells,
                   "particles": n_part, "nx_nz": "from {64,128,256,512}", "alpha": "U[0.3,0.7]",
                   "gamma": "{10,50,130}", "shape": "linear galerkin", "correction": "Psi_E/Psi_B quartic",
                   "filter": "4-pass 1-2-1 per axis", "schedule": "batched hipGraph"},
        "plain_eager_particle_steps_per_s": n_part * K / b["plain_eager_s"],
        "plain_graph_particle_steps_per_s": n_part * K / b["plain_graph_s"],
        "speedup_batched_vs_plain_eager": b["plain_eager_s"] / b["batched_s"],
        "speedup_batched_vs_plain_graph": b["plain_graph_s"] / b["batched_s"],
        "adjoint_cost_ratio": None if adj is None else adj["ratio"],
        "grid_cell_updates_per_s": n_cells * K / b["batched_s"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
                     "kernel": "k_particles<2,1,float> (batched launch)", "bytes_per_launch": pk_bytes,
                     "avg_launch_ms": pk_ms},
        "roofline_step": {"bound": "hbm", "achieved": sb / (ms_step * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": sb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_step": sb, "bytes_per_particle_step": sb / n_part},
        "kernels_ms": b["kernels_ms"],
        "tuning": b["tuning"],
        "particle_kernel_valu": valu_issue("batched64_fp32", n_part, pk_ms),
        "gauss_linf_rel_max": b["gauss_linf_rel_max"],
        "kernel_profile_before_timing_steps": 2 * args.profile_steps,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "kernel_source_sha": kernel_sha(),
    }
    if args.extra:
        out["extra"] = extra_blocks()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
