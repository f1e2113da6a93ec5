"""Write the FP64 oracle's transverse field-energy traces used as growth-rate goldens.

Usage: python tests/golden/make_growth_golden.py [--workers N] [--only PREFIX]

Calls only oracle/ (and the seeded inputs of pic_inputs).  One serial oracle
process per instance; instances run in parallel worker processes, longest
first.  Cases:
  c1     512x512, 16 ppc, correction + 4-pass filter, alpha 0.3 / 0.5 / 0.7,
         2000 steps (pic_inputs.growth_cases)
  c3     the 64-instance batch: the first 64 entries of
         pic_inputs.batched_candidates(0) whose correction the oracle accepts
         (Psi_B > 0 on [0, 1], Psi_E > 0 on [0, 1)), 1000 steps each
  scan   the Sec. 3 setting at 64x64, 8 ppc (gamma x alpha, correction on/off)
  var    the Sec. 3 / Sec. 4 variants of that setting
For each instance the trace W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV after
steps 1..N and the initial kinetic energy are stored:
  tests/golden/growth_oracle.npz   traces (float64), one array per key
  tests/golden/growth_oracle.json  per key: workload, seed, steps, Wkin(0), and
                                   the oracle fit's growth rate and window
Intermediate results go to tests/golden/_growth_parts/ (removed at the end),
so an interrupted run resumes.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import pic_inputs as pi  # noqa: E402
from oracle import fit as ofit  # noqa: E402
from oracle import psi as opsi  # noqa: E402

PARTS = os.path.join(HERE, "_growth_parts")


def oracle_accepts(wl):
    if not wl.get("correction"):
        return True
    a, b, _ = opsi.psi_coeffs(wl.get("interp", "galerkin"), wl["alpha"])
    return opsi.psi_positive(a, b)


def batch_cases():
    out = []
    for i, cand in enumerate(pi.batched_candidates(0)):
        if oracle_accepts(cand):
            out.append(("c3_%03d" % i, cand, cand["seeds"][0], cand["steps"]))
        if len(out) == 64:
            break
    return out


def run_case(case):
    key, wl, seed, steps = case
    path = os.path.join(PARTS, key + ".npz")
    if os.path.exists(path):
        return key
    from oracle.ref import OracleSim
    x, u = pi.load_beam(wl["dims"], wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], seed)
    sim = OracleSim(wl, x, u)
    wkin0 = sim.energies()["Wkin"]
    del x, u
    W = np.empty(steps)
    t0 = time.time()
    for n in range(steps):
        sim.step(1)
        W[n] = 0.5 * sim.dV * float(np.sum(sim.E[0] ** 2) + np.sum(sim.E[1] ** 2) +
                                    np.sum(sim.B[0] ** 2) + np.sum(sim.B[1] ** 2))
    np.savez(path + ".tmp.npz", W=W, wkin0=wkin0, status=sim.status)
    os.replace(path + ".tmp.npz", path)
    print("%s done in %.0f s (status %d)" % (key, time.time() - t0, sim.status), flush=True)
    return key


def cost(case):
    _, wl, _, steps = case
    return wl["ppc"] * int(np.prod(wl["n"])) * steps * (8 if wl["order"] == 3 else 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    os.makedirs(PARTS, exist_ok=True)
    cases = [c for c in pi.growth_cases() + batch_cases() if c[0].startswith(args.only)]
    todo = sorted(cases, key=cost, reverse=True)
    print("%d cases, %d workers" % (len(todo), args.workers), flush=True)
    with mp.get_context("fork").Pool(args.workers) as pool:
        for _ in pool.imap_unordered(run_case, todo):
            pass
    traces, meta = {}, {}
    for key, wl, seed, steps in cases:
        d = np.load(os.path.join(PARTS, key + ".npz"))
        W, wkin0 = d["W"], float(d["wkin0"])
        g, win = ofit.growth_rate(list(W), wl["alpha"], wkin0)
        traces[key] = W
        meta[key] = {"workload": {k: (list(v) if isinstance(v, tuple) else v) for k, v in wl.items()},
                     "seed": seed, "steps": steps, "wkin0": wkin0, "status": int(d["status"]),
                     "gamma_fit": g, "window": list(win)}
    if args.only:
        print(json.dumps({k: (m["gamma_fit"], m["window"]) for k, m in meta.items()}, indent=1))
        return
    np.savez_compressed(os.path.join(HERE, "growth_oracle.npz"), **traces)
    with open(os.path.join(HERE, "growth_oracle.json"), "w") as f:
        json.dump({"source": "tests/golden/make_growth_golden.py (FP64 C oracle, serial per instance)",
                   "trace": "W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV after steps 1..N",
                   "cases": meta}, f, indent=1)
    for key, *_ in cases:
        os.remove(os.path.join(PARTS, key + ".npz"))
    os.rmdir(PARTS)


if __name__ == "__main__":
    main()
