"""Benchmark of the GPU PIC step on one MI355X.

Workload: 2D 512x512 periodic Yee grid, 16 particles per cell (4,194,304
macro-particles), cold beam gamma = 130 along z with 1e-4 relative momentum
spread, c dt / dz = 0.5, linear Galerkin shapes, correction stencils (Psi_E /
Psi_B, quartics) plus a 4-pass (1,2,1) filter per axis, FP32 particles and
fields (int32 cell index + FP32 offset, fixed-point current).  Synthetic
seeded input (pic_inputs).

A step is the whole hot path: Yee update, fields as seen by the particles
(correction + filter), gather, Boris push, move, Esirkepov deposit, and the
periodic tile re-sort check.  `value` = particle-steps per second over the
timed steps (inputs resident in HBM, HIP-graph replay).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extra]
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1401_0838_amd", "csrc", "pic_kernels.hip")


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def particle_kernel_bytes(n_particles, n_cells, word=4, state_bytes=24):
    """Algorithmic HBM bytes of one particle-kernel launch: every particle's state read
    and written once (state_bytes each way), the six seen-field components read once
    and the three current components written once per cell."""
    return 2 * state_bytes * n_particles + 9 * word * n_cells


def stored_traffic(name):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel source; else None."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    if doc.get("kernel_source_sha") != kernel_sha():
        return None
    return doc.get("hbm_bytes_per_launch")


VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock (no packed FP32)


def valu_issue(case, n_part, launch_ms):
    """Fraction of the vector-ALU issue ceiling a particle-kernel launch reaches:
    lane instructions per particle from committed SQ_INSTS_VALU counter runs
    (only if they were taken on the current kernel source) times the particles,
    over the measured launch duration."""
    path = os.path.join(PROFILE_DIR, "valu_k_particles.json")
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    if doc.get("kernel_source_sha") != kernel_sha() or case not in doc.get("cases", {}):
        return None
    per = doc["cases"][case]["valu_lane_instr_per_particle"]
    achieved = per * n_part / (launch_ms * 1e-3)
    return {"bound": "alu", "valu_lane_instr_per_particle": per, "achieved": achieved / 1e12,
            "peak": VALU_PEAK_LANE_INSTR / 1e12, "unit": "T lane-instr/s", "frac": achieved / VALU_PEAK_LANE_INSTR}


def cpu_baseline(wl, x, u, steps):
    """The FP64 oracle (single thread, as it stands) on a bounded sample: `steps`
    steps of the same 512x512, 16 ppc workload."""
    from oracle.ref import OracleSim
    ref = OracleSim(wl, x, u)
    t0 = time.perf_counter()
    ref.step(steps)
    dt = time.perf_counter() - t0
    return {"value": x.shape[0] * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the full 512x512 x 16 ppc workload, FP64 C oracle, 1 thread, %.1f s"
                      % (steps, dt)}


def batched_block(steps, warmup):
    """64 uneven 2D instances (nx, nz in {64..512}, alpha in [0.3, 0.7], gamma in
    {10, 50, 130}, 8 ppc, FP32): batched graph-replayed step vs one launch per
    instance per kernel, same kernels, same GPU."""
    import pic_inputs as pi
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd.sim import Simulation
    wls, parts = [], []
    for cand in pi.batched_candidates(0):
        rc, _, _ = L.pic_psi_coeffs(L.PIC_GALERKIN, cand["alpha"], 4)
        if rc != L.PIC_OK:
            continue
        wls.append(cand)
        parts.append(pi.load_beam(2, cand["n"], cand["ppc"], cand["gamma"], cand["sigma"], cand["seeds"][0]))
        if len(wls) == 64:
            break
    n_part = sum(p[0].shape[0] for p in parts)
    out = {"instances": len(wls), "particles": n_part,
           "cells": sum(w["n"][0] * w["n"][1] for w in wls)}
    for sched, graph in (("batched", True), ("plain", False)):
        sim = Simulation(wls, parts, precision="fp32")
        sim.set_schedule(sched, graph)
        sim.step(warmup)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        dt = time.perf_counter() - t0
        if sched == "batched":
            prof = sim.profile(10)
            out["batched_particle_ms"] = prof["particle_ms"]
            out["batched_bytes_per_particle_launch"] = particle_kernel_bytes(n_part, out["cells"])
        sim.close()
        out[sched + "_particle_steps_per_s"] = n_part * steps / dt
        out[sched + "_ms_per_step"] = 1e3 * dt / steps
        out[sched + "_grid_cell_updates_per_s"] = out["cells"] * steps / dt
    out["speedup_batched_vs_plain"] = out["batched_particle_steps_per_s"] / out["plain_particle_steps_per_s"]
    out["batched_hbm_frac"] = (out["batched_bytes_per_particle_launch"] / (out["batched_particle_ms"] * 1e-3)
                               / 1e9 / HBM_PEAK_GBS)
    return out


def beam3d_block(steps, warmup):
    """3D 128x128x256, 8 ppc (33.5M particles), cubic shapes, correction + filter,
    FP32: particle-steps/s and the particle kernel's HBM fraction (this case is
    bound by VALU and LDS atomics, not HBM: ~250 gathered nodes and 300 current
    updates per particle)."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    wl = pi.workload("beam3d_128x128x256")
    x, u = pi.load_beam(3, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    sim = Simulation(wl, (x, u), precision="fp32")
    n_part = x.shape[0]
    n_cells = wl["n"][0] * wl["n"][1] * wl["n"][2]
    del x, u
    sim.step(warmup)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt = time.perf_counter() - t0
    prof = sim.profile(5)
    d = sim.diag()
    sim.close()
    pk = particle_kernel_bytes(n_part, n_cells, state_bytes=28)
    return {"particles": n_part, "cells": n_cells, "particle_steps_per_s": n_part * steps / dt,
            "grid_cell_updates_per_s": n_cells * steps / dt,
            "ms_per_step": 1e3 * dt / steps, "kernels_ms": {k: prof[k] for k in ("yee_ms", "seen_ms", "particle_ms")},
            "particle_kernel_hbm_frac": pk / (prof["particle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "particle_kernel_valu": valu_issue("beam3d_128x128x256_ppc8_cubic_fp32", n_part, prof["particle_ms"]),
            "gauss_linf_rel": d["gauss_linf"] / max(d["rho_max"], 1e-300), "slow_tiles": d["slow_tiles"]}


def fp64_block(steps, warmup):
    """The 512x512, 16 ppc step in FP64 (44 B of particle state, FP64 current):
    particle-steps/s and the particle kernel's HBM fraction."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    wl = pi.workload("beam2d_512", alpha=0.5, precision="fp64")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    sim = Simulation(wl, (x, u), precision="fp64")
    n_part, n_cells = x.shape[0], wl["n"][0] * wl["n"][1]
    sim.step(warmup)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt = time.perf_counter() - t0
    prof = sim.profile(5)
    sim.close()
    pk = particle_kernel_bytes(n_part, n_cells, word=8, state_bytes=44)
    return {"particle_steps_per_s": n_part * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "particle_kernel_ms": prof["particle_ms"],
            "particle_kernel_hbm_frac": pk / (prof["particle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}


def schemes_block(steps, warmup):
    """The 512x512, 16 ppc FP32 step with the Uniform (Eq. 4) and
    momentum-conserving (Eq. 5) gathers, and with the exact Psi_E / Psi_B on the
    transverse E (Galerkin gather; the seen-field time includes the inversion
    along z): particle-steps/s, per-kernel times and the particle kernel's HBM
    fraction (same algorithmic bytes as Galerkin: the gathers read the same
    staged window)."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    out = {}
    for interp, corr in (("uniform", True), ("momentum", True), ("galerkin", "ratio")):
        wl = pi.workload("beam2d_512", alpha=0.5, precision="fp32", interp=interp, correction=corr)
        x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
        sim = Simulation(wl, (x, u), precision="fp32")
        sim.set_schedule("batched", True)
        n_part, n_cells = x.shape[0], wl["n"][0] * wl["n"][1]
        sim.step(warmup)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        dt = time.perf_counter() - t0
        prof = sim.profile(10)
        sim.close()
        pk = particle_kernel_bytes(n_part, n_cells)
        key = interp if corr is True else "exact_ratio"
        out[key] = {"particle_steps_per_s": n_part * steps / dt, "ms_per_step": 1e3 * dt / steps,
                       "kernels_ms": {k: prof[k] for k in ("yee_ms", "seen_ms", "particle_ms", "step_ms")},
                       "particle_kernel_hbm_frac": pk / (prof["particle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def ck_block(steps, warmup):
    """Cole-Karkkainen solver (2D, beta = 1/8), FP32: the 512x512 x 16 ppc step at
    alpha = 0.9 (above the Yee limit 1/sqrt(2)), and the Sec. 3 setting
    (128x128 x 16 ppc, cubic shapes, Eq. 6 filter, correction, alpha = 0.9)."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    out = {}
    cases = (("beam2d_512_alpha0.9", pi.workload("beam2d_512", alpha=0.9, solver="ck")),
             ("beam2d_128_cubic_eq6", pi.workload("beam2d_128_ck")))
    for name, wl in cases:
        x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
        sim = Simulation(wl, (x, u), precision="fp32")
        sim.set_schedule("batched", True)
        n_part, n_cells = x.shape[0], wl["n"][0] * wl["n"][1]
        sim.step(warmup)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        dt = time.perf_counter() - t0
        prof = sim.profile(10)
        sim.close()
        pk = particle_kernel_bytes(n_part, n_cells)
        out[name] = {"particles": n_part, "particle_steps_per_s": n_part * steps / dt,
                     "ms_per_step": 1e3 * dt / steps,
                     "kernels_ms": {k: prof[k] for k in ("yee_ms", "seen_ms", "particle_ms", "step_ms")},
                     "particle_kernel_hbm_frac": pk / (prof["particle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def gamma_scan_block(steps):
    """Sec. 3 growth-rate scan through the batched engine: the 128x128 x 16 ppc
    cubic CK setting with the Eq. 6 filter, gamma in {3, 10, 30, 130} x alpha in
    {0.3 .. 0.99}, with and without the correction, FP32, `steps` steps per batch.
    Reports the scan's throughput, each gamma's peak growth rate and the fitted
    power of gamma (the paper reads about -1/2 for its peaks)."""
    import pic_inputs as pi
    from paper_1401_0838_amd import scan
    alphas = [0.3, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99]
    gammas = [3.0, 10.0, 30.0, 130.0]
    out = {"workload": "beam2d_128_ck (128x128, 16 ppc, cubic, CK, Eq. 6 filter)", "steps": steps,
           "alphas": alphas, "gammas": gammas}
    for corr in (True, False):
        base = pi.workload("beam2d_128_ck", correction=corr)
        pts, wls, parts, skipped = scan.scan_instances(base, alphas, gammas)
        n_part = sum(p[0].shape[0] for p in parts)
        t0 = time.perf_counter()
        traces, wkin = scan.run_scan(pts, wls, parts, steps, "fp32")
        dt = time.perf_counter() - t0
        rates, peaks, power = scan.growth_table(pts, traces, wkin)
        key = "corrected" if corr else "uncorrected"
        out[key] = {"instances": len(pts), "skipped": skipped,
                    "particle_steps_per_s": n_part * steps / dt, "wall_s": dt,
                    "growth_rates": {"%g/%g" % p: r for p, r in zip(pts, rates)},
                    "peak_growth": {"%g" % g: {"rate": v[0], "alpha": v[1]} for g, v in sorted(peaks.items())},
                    "peak_power_of_gamma": power}
    return out


def variants_block(steps):
    """Sec. 3's variants of its setting (128x128 x 16 ppc cubic CK, Eq. 6 filter,
    correction): no filter apart from Psi_B, the exact Psi_E / Psi_B on the
    transverse E only, no compensation passes; growth rates at gamma = 130 and
    3 over alpha, and each variant's rate over the baseline's (the paper reads
    about 2x, 3x and 'moderately lower' at large alpha)."""
    import pic_inputs as pi
    from paper_1401_0838_amd import scan
    alphas = [0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99]
    out = {"workload": "beam2d_128_ck (128x128, 16 ppc, cubic, CK, Eq. 6 filter)", "steps": steps,
           "alphas": alphas}
    for gamma in (130.0, 3.0):
        t0 = time.perf_counter()
        rates, skipped = scan.variant_sweep(pi.workload("beam2d_128_ck"), alphas, gamma, steps)
        base = rates["baseline"]
        out["gamma_%g" % gamma] = {
            "wall_s": time.perf_counter() - t0, "skipped": skipped, "growth_rates": rates,
            "over_baseline": {k: [None if (x is None or y in (None, 0)) else x / y for x, y in zip(v, base)]
                              for k, v in rates.items() if k != "baseline"}}
    return out


def adjoint_block():
    """256x256, 8 ppc, 200 steps, checkpoints every 20 (FP32): backward (recompute +
    reverse sweep) time over forward time."""
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation
    wl = pi.workload("beam2d_256_adjoint")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    n = wl["steps"]
    fwd = Simulation(wl, (x, u), precision="fp32")
    fwd.step(5)
    fwd.synchronize()
    t0 = time.perf_counter()
    fwd.step(n)
    fwd.synchronize()
    t_step = time.perf_counter() - t0
    fwd.close()
    sim = Simulation(wl, (x, u), precision="fp32", adjoint_steps=n, adjoint_ckpt=wl["checkpoint"])
    t0 = time.perf_counter()
    sim.adjoint_forward(n)
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.adjoint_backward()
    t_b = time.perf_counter() - t0
    sim.close()
    return {"steps": n, "checkpoint_every": wl["checkpoint"], "forward_s": t_step,
            "forward_with_checkpoints_s": t_f, "backward_s": t_b, "ratio": t_b / t_step}


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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance batched comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost ratio")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D cubic case")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 512x512 case")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the Uniform and momentum-conserving gather cases")
    ap.add_argument("--no-ck", action="store_true", help="skip the Cole-Karkkainen solver cases")
    ap.add_argument("--no-scan", action="store_true", help="skip the gamma / alpha growth-rate scan")
    ap.add_argument("--no-variants", action="store_true", help="skip the Sec. 3 variant growth rates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--only", choices=("batched", "adjoint", "3d", "fp64", "schemes", "ck", "scan", "variants"),
                    help="run one secondary block alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only:
        blk = {"batched": lambda: batched_block(max(20, args.steps // 4), 5), "adjoint": adjoint_block,
               "3d": lambda: beam3d_block(20, 3), "fp64": lambda: fp64_block(50, 5),
               "schemes": lambda: schemes_block(100, 10), "ck": lambda: ck_block(100, 10),
               "scan": lambda: gamma_scan_block(2000), "variants": lambda: variants_block(2000)}[args.only]()
        print(json.dumps({args.only: blk}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(batches would shard by instance; one large domain along z in slabs, with guard-layer "
              "exchange of E, B and J and particle migration across slab faces)", file=sys.stderr)
        sys.exit(2)

    import torch
    import pic_inputs as pi
    from paper_1401_0838_amd.sim import Simulation

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = pi.workload("beam2d_512", alpha=0.5, precision="fp32")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    sim = Simulation(wl, (x, u), precision="fp32")
    sim.set_schedule("batched", True)
    n_part = x.shape[0]
    n_cells = wl["n"][0] * wl["n"][1]

    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n_part * args.steps / elapsed

    # per-kernel durations with HIP events on the library's stream
    prof = sim.profile(args.profile_steps)
    d = sim.diag()
    sim.close()
    pk_bytes = particle_kernel_bytes(n_part, n_cells)
    achieved = pk_bytes / (prof["particle_ms"] * 1e-3) / 1e9
    traffic = stored_traffic("traffic_k_particles_beam2d_512_fp32.json")
    out = {
        "metric": "particle-steps/s (gather+Boris+Esirkepov) plain vs batched; adjoint cost ratio",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "beam2d_512x512_ppc16_fp32", "cells": n_cells, "particles": n_part,
                   "alpha": 0.5, "gamma": 130.0, "shape": "linear galerkin",
                   "correction": "Psi_E/Psi_B quartic", "filter": "4-pass 1-2-1 per axis",
                   "schedule": "batched hipGraph"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_particles<2,1,float>", "bytes_per_launch": pk_bytes,
                     "avg_launch_ms": prof["particle_ms"]},
        "kernels_ms": {k: prof[k] for k in ("yee_ms", "seen_ms", "particle_ms", "resort_ms", "step_ms")},
        "particle_kernel_valu": valu_issue("beam2d_512x512_ppc16_fp32", n_part, prof["particle_ms"]),
        "grid_cell_updates_per_s": n_cells * args.steps / elapsed,
        "gauss_linf_rel": d["gauss_linf"] / max(d["rho_max"], 1e-300),
        "kernel_source_sha": kernel_sha(),
    }
    if not args.no_batched:
        out["batched"] = batched_block(max(20, args.steps // 4), 5)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_block()
    if not args.no_3d:
        out["beam3d"] = beam3d_block(20, 3)
    if not args.no_fp64:
        out["beam2d_fp64"] = fp64_block(50, 5)
    if not args.no_schemes:
        out["schemes"] = schemes_block(100, 10)
    if not args.no_ck:
        out["ck"] = ck_block(100, 10)
    if not args.no_scan:
        out["gamma_scan"] = gamma_scan_block(2000)
    if not args.no_variants:
        out["variants"] = variants_block(2000)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, x, u, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
