"""Growth-rate scans through the batched engine (Sec. 3, Figs. 2-3, and the
variants Sec. 3 compares).

Sec. 3 plots the maximum growth rate of the numerical instability against
c dt / dz for gamma = 130 and gamma = 3, and reads the peak growth rates as
scaling very roughly like gamma^(-1/2).  A scan here is one batch of
instances, one per (gamma, alpha) point, stepped together on the GPU with a
per-step trace of the transverse field energy; each trace gives a growth rate
(fit.growth_rate), each gamma its peak over alpha, and the peaks a fitted
power of gamma.  Points whose correction polynomials break down (pic_psi_coeffs
returns PIC_EPSI; Sec. 3 excises such a window) are skipped and reported.
"""
import math

import numpy as np

from . import _lib as L
from . import fit


def scan_instances(base, alphas, gammas, seed=0):
    """Workloads and seeded beams for every accepted (gamma, alpha) point.

    base   : workload dict (grid, shapes, solver, filter, correction, ppc ...)
    Returns (points, workloads, particles, skipped) with points[i] = (gamma, alpha).
    """
    import pic_inputs as pi
    interp = {"galerkin": L.PIC_GALERKIN, "uniform": L.PIC_UNIFORM,
              "momentum": L.PIC_MOMENTUM}[base.get("interp", "galerkin")]
    points, wls, parts, skipped = [], [], [], []
    for gi, gamma in enumerate(gammas):
        for ai, alpha in enumerate(alphas):
            if base.get("correction"):
                rc, _, _ = L.pic_psi_coeffs(interp, float(alpha), 4)
                if rc != L.PIC_OK:
                    skipped.append((gamma, alpha))
                    continue
            wl = dict(base, alpha=float(alpha), gamma=float(gamma), name="scan_g%g_a%g" % (gamma, alpha))
            x, u = pi.load_beam(wl["dims"], wl["n"], wl["ppc"], wl["gamma"], wl["sigma"],
                                seed + 1000 * gi + ai)
            points.append((float(gamma), float(alpha)))
            wls.append(wl)
            parts.append((x, u))
    return points, wls, parts, skipped


def run_scan(points, wls, parts, nsteps, precision="fp32", info=None):
    """Step every instance nsteps in one batched run (tile, launch options and
    schedule from the autotuner's cache when it has the batch); return the
    transverse field-energy traces (list of arrays) and each instance's initial
    kinetic energy.  info (a dict), if given, collects the tuner's picks."""
    from .sim import Simulation
    sim = Simulation(wls, parts, precision=precision, trace_capacity=nsteps, tuned=True)
    if info is not None:
        info.setdefault("tuning", []).append(sim.tuning)
    try:
        wkin = [sim.diag(i)["Wkin"] for i in range(len(wls))]
        sim.step(nsteps)
        traces = []
        for i in range(len(wls)):
            tr = sim.trace(i)
            traces.append(tr[:, 0] + tr[:, 1] + tr[:, 3] + tr[:, 4])
    finally:
        sim.close()
    return traces, wkin


def growth_table(points, traces, wkin):
    """Growth rate per point, peak over alpha per gamma, and the least-squares
    power p of peak ~ gamma^p (None with fewer than two positive peaks)."""
    rates = [fit.growth_rate(W, alpha, wk)[0] for (gamma, alpha), W, wk in zip(points, traces, wkin)]
    peaks = {}
    for (gamma, alpha), g in zip(points, rates):
        if gamma not in peaks or g > peaks[gamma][0]:
            peaks[gamma] = (g, alpha)
    gs = sorted(g for g in peaks if peaks[g][0] > 0)
    power = None
    if len(gs) >= 2:
        power = float(np.polyfit([math.log(g) for g in gs], [math.log(peaks[g][0]) for g in gs], 1)[0])
    return rates, peaks, power


# Sec. 3's variants of its Fig. 2 setting (correction, Eq. 6 filter): (1) no
# digital filtering apart from Psi_B; (2) Psi_E / Psi_B applied to the
# transverse E only (Psi_B inverted); (3) no compensation passes; and Sec. 4's
# filter with one bilinear and one compensation pass (the square root of Eq. 6)
def _variants():
    import pic_inputs as pi
    return dict(pi.VARIANTS)


VARIANTS = _variants()


def variant_batches(base, alphas, gamma, seed=0):
    """The batches of a variant sweep: variants that share the split correction
    form one, the exact-ratio one another (a batch shares that choice).  Yields
    (points, workloads, particles, variant of each instance, skipped points)."""
    groups = {}
    for name, over in VARIANTS.items():
        groups.setdefault(over["correction"] == "ratio", []).append(name)
    for names in groups.values():
        pts, wls, parts, tags, skipped = [], [], [], [], []
        for name in names:
            p, w, pa, sk = scan_instances(dict(base, **VARIANTS[name]), alphas, [gamma], seed)
            pts += p
            wls += w
            parts += pa
            tags += [name] * len(p)
            skipped += [(name,) + k for k in sk]
        yield pts, wls, parts, tags, skipped


def variant_sweep(base, alphas, gamma, nsteps, precision="fp32", seed=0, info=None):
    """Growth rate of every variant at every alpha (one gamma).  Variants that
    share the split correction run as one batch; the exact-ratio one as another
    (a batch shares that choice).  Returns {variant: [rate per alpha]} and the
    points skipped for a broken-down correction."""
    rates, skipped = {}, []
    for pts, wls, parts, tags, sk in variant_batches(base, alphas, gamma, seed):
        skipped += sk
        traces, wkin = run_scan(pts, wls, parts, nsteps, precision, info)
        r, _, _ = growth_table(pts, traces, wkin)
        for name, (g, a), v in zip(tags, pts, r):
            rates.setdefault(name, {})[a] = v
    return {name: [rates[name].get(float(a)) for a in alphas] for name in VARIANTS}, skipped
