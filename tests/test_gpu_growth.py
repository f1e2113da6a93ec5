"""Instability growth rates: GPU (FP32 and FP64) against the FP64 oracle.

Growth rate of the transverse field energy (fit window and definition in
paper_1401_0838_amd/fit.py; the oracle side uses its own oracle/fit.py).
Bar: within 5 %, or |dGamma| dt <= 5e-5 when the growth is too weak for a
relative comparison (Gamma dt < 1e-4 or less than ten-fold total growth).
"""
import sys

import numpy as np
import pytest

import pic_inputs as pi
from oracle import fit as ofit
from oracle.ref import OracleSim
from paper_1401_0838_amd import fit as gfit

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_trace(wl, x, u, prec, nsteps):
    from paper_1401_0838_amd.sim import Simulation
    sim = Simulation(wl, (x, u), precision=prec, trace_capacity=nsteps)
    wkin0 = sim.diag()["Wkin"]
    sim.step(nsteps)
    tr = sim.trace()
    sim.close()
    W = tr[:, 0] + tr[:, 1] + tr[:, 3] + tr[:, 4]
    return W, wkin0


def _oracle_trace(wl, x, u, nsteps):
    ref = OracleSim(wl, x, u)
    wkin0 = ref.energies()["Wkin"]
    W = []
    for _ in range(nsteps):
        ref.step(1)
        W.append(ref.energies()["Wperp"])
    return np.array(W), wkin0


def _close(g_a, g_b, W, dt):
    weak = abs(g_b) * dt < 1e-4 or W.max() < 10 * max(W[W > 0].min(), 1e-300)
    if weak:
        return abs(g_a - g_b) * dt <= 5e-5
    return abs(g_a - g_b) <= 0.05 * abs(g_b)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_growth_rate_plain_method_vs_oracle(alpha):
    """No correction, no filter: the instability grows fast; the GPU trace and the
    fitted rate follow the oracle."""
    wl = pi.workload("beam2d_64_fp64", alpha=alpha)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    n = 400
    Wo, wk = _oracle_trace(wl, x, u, n)
    go, _ = ofit.growth_rate(list(Wo), wl["alpha"], wk)
    for prec in ("fp64", "fp32"):
        Wg, wkg = _gpu_trace(wl, x, u, prec, n)
        gg, win = gfit.growth_rate(Wg, wl["alpha"], wkg)
        _say("alpha %.1f %s: Gamma gpu %.6e oracle %.6e window %s" % (alpha, prec, gg, go, win))
        assert len(Wg) == n
        if prec == "fp64":
            assert np.max(np.abs(Wg - Wo)) < 1e-9 * np.max(Wo)
        assert _close(gg, go, Wo, wl["alpha"])


def test_growth_rate_corrected_vs_oracle():
    """Correction + 4-pass filter (the 512x512 configuration's method at 64x64)."""
    wl = pi.workload("beam2d_512", n=(64, 64), ppc=4, alpha=0.5)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    n = 400
    Wo, wk = _oracle_trace(wl, x, u, n)
    go, _ = ofit.growth_rate(list(Wo), wl["alpha"], wk)
    Wg, wkg = _gpu_trace(wl, x, u, "fp32", n)
    gg, _ = gfit.growth_rate(Wg, wl["alpha"], wkg)
    _say("corrected: Gamma gpu %.6e oracle %.6e" % (gg, go))
    assert _close(gg, go, Wo, wl["alpha"])


def test_growth_rate_full_size_fp32_vs_fp64():
    """512x512, 16 ppc, 2000 steps at alpha 0.3, 0.5, 0.7: the FP32 growth rate equals
    the FP64 one (a property that holds at any size; the oracle is checked at 64x64)."""
    wl0 = pi.workload("beam2d_512")
    x, u = pi.load_beam(2, wl0["n"], wl0["ppc"], wl0["gamma"], wl0["sigma"], 0)
    for alpha in wl0["alphas"]:
        wl = dict(wl0, alpha=alpha)
        W64, wk = _gpu_trace(wl, x, u, "fp64", wl["steps"])
        W32, _ = _gpu_trace(wl, x, u, "fp32", wl["steps"])
        g64, win = gfit.growth_rate(W64, alpha, wk)
        g32, _ = gfit.growth_rate(W32, alpha, wk)
        _say("512 alpha %.1f: Gamma fp32 %.6e fp64 %.6e (Gamma dt %.2e) window %s W %.3e..%.3e"
             % (alpha, g32, g64, g64 * alpha, win, W64[10], W64[-1]))
        assert _close(g32, g64, W64, alpha)


def test_batched_scan_growth_rates_fp32_vs_fp64():
    """The 64-instance scan (uneven grids, alpha in [0.3, 0.7], gamma in {10, 50,
    130}, 8 ppc), 1000 steps in one batched run per precision: every instance's
    FP32 growth rate equals its FP64 one (same bar).  Candidates whose
    correction breaks down are skipped and counted."""
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd.sim import Simulation
    wls, parts, skipped = [], [], 0
    for cand in pi.batched_candidates(0):
        rc, _, _ = L.pic_psi_coeffs(L.PIC_GALERKIN, cand["alpha"], 4)
        if rc != L.PIC_OK:
            skipped += 1
            continue
        wls.append(cand)
        parts.append(pi.load_beam(2, cand["n"], cand["ppc"], cand["gamma"], cand["sigma"], cand["seeds"][0]))
        if len(wls) == 64:
            break
    nsteps = wls[0]["steps"]
    traces, wkin = {}, {}
    for prec in ("fp32", "fp64"):
        sim = Simulation(wls, parts, precision=prec, trace_capacity=nsteps)
        wkin[prec] = [sim.diag(i)["Wkin"] for i in range(len(wls))]
        sim.step(nsteps)
        traces[prec] = []
        for i in range(len(wls)):
            tr = sim.trace(i)
            traces[prec].append(tr[:, 0] + tr[:, 1] + tr[:, 3] + tr[:, 4])
        sim.close()
    _say("batched scan: %d instances, %d candidates skipped for a broken-down correction" % (len(wls), skipped))
    bad = []
    for i, w in enumerate(wls):
        W32, W64 = traces["fp32"][i], traces["fp64"][i]
        assert len(W32) == nsteps and len(W64) == nsteps
        g32, _ = gfit.growth_rate(W32, w["alpha"], wkin["fp64"][i])
        g64, _ = gfit.growth_rate(W64, w["alpha"], wkin["fp64"][i])
        if not _close(g32, g64, W64, w["alpha"]):
            bad.append((i, w["n"], w["alpha"], w["gamma"], g32, g64))
    _say("  mismatches: %s" % bad)
    assert not bad


def test_growth_rate_ck_cubic_eq6_vs_oracle():
    """The Sec. 3 setting (cubic, CK, Eq. 6 filter, correction) at 32x32, 4 ppc,
    alpha = 0.9: the GPU traces follow the oracle and the fitted rates agree."""
    wl = pi.workload("beam2d_128_ck", n=(32, 32), ppc=4, alpha=0.9, correction=True)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    n = 400
    Wo, wk = _oracle_trace(wl, x, u, n)
    go, _ = ofit.growth_rate(list(Wo), wl["alpha"], wk)
    for prec in ("fp64", "fp32"):
        Wg, wkg = _gpu_trace(wl, x, u, prec, n)
        gg, win = gfit.growth_rate(Wg, wl["alpha"], wkg)
        _say("ck cubic eq6 %s: Gamma gpu %.6e oracle %.6e window %s" % (prec, gg, go, win))
        if prec == "fp64":
            assert np.max(np.abs(Wg - Wo)) < 1e-9 * np.max(Wo)
        assert _close(gg, go, Wo, wl["alpha"])


def test_gamma_scan_growth_rates_fp32_vs_fp64():
    """A gamma x alpha scan at the Sec. 3 setting (64x64, 8 ppc, cubic, CK, Eq. 6
    filter; gamma 3 and 130, alpha 0.5 and 0.9, with and without correction),
    1000 steps in one batched run per precision: every FP32 growth rate equals
    its FP64 one (same bar)."""
    from paper_1401_0838_amd import scan
    bad = []
    for corr in (True, False):
        base = pi.workload("beam2d_128_ck", n=(64, 64), ppc=8, correction=corr)
        pts, wls, parts, skipped = scan.scan_instances(base, [0.5, 0.9], [3.0, 130.0])
        tr32, wk32 = scan.run_scan(pts, wls, parts, 1000, "fp32")
        tr64, wk64 = scan.run_scan(pts, wls, parts, 1000, "fp64")
        r32, _, _ = scan.growth_table(pts, tr32, wk64)
        r64, peaks, power = scan.growth_table(pts, tr64, wk64)
        _say("gamma scan corr=%s: fp64 rates %s peaks %s power %s" % (corr, r64, peaks, power))
        for p, g32, g64, W in zip(pts, r32, r64, tr64):
            if not _close(g32, g64, W, p[1]):
                bad.append((corr, p, g32, g64))
    _say("  mismatches: %s" % bad)
    assert not bad


def test_variant_sweep_growth_rates_fp32_vs_fp64():
    """Sec. 3's variants (no filter, exact ratio on the transverse E, no
    compensation) at 64x64, 8 ppc, cubic CK, gamma 130, alpha 0.7 and 0.95,
    1000 steps: FP32 growth rates equal FP64 ones for every variant."""
    from paper_1401_0838_amd import scan
    base = pi.workload("beam2d_128_ck", n=(64, 64), ppc=8)
    r32, _ = scan.variant_sweep(base, [0.7, 0.95], 130.0, 1000, "fp32")
    r64, _ = scan.variant_sweep(base, [0.7, 0.95], 130.0, 1000, "fp64")
    _say("variants fp32 %s\n         fp64 %s" % (r32, r64))
    for name in r64:
        for g32, g64, a in zip(r32[name], r64[name], (0.7, 0.95)):
            assert abs(g32 - g64) <= 0.05 * abs(g64) or abs(g32 - g64) * a <= 5e-5, (name, a, g32, g64)
